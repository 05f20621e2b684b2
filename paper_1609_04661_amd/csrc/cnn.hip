// Residual CNN denoiser D(r) = r - f(r) on MFMA (the learned plug-in; the
// method treats the denoiser as a black box, Sec. 4.3), its forward-mode
// tangent for the Monte-Carlo divergence (eq. MC_SURE in the eps -> 0 limit:
// b^T J_D b = b^T b - b^T J_f b), and the training kernels (MSE loss,
// backward, Adam).
//
// f = conv(1->64) ReLU, 8 x [conv(64->64) ReLU], conv(64->1); 3x3, bias,
// zero padding, cross-correlation.  Activations are BF16 NHWC (64 channels
// contiguous per pixel); the 64->64 layers are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   M = 16 output channels, N = 16 pixels of one tile row, K = 32 input
//   channels of one tap; 9 taps x 2 channel halves = 18 K-steps.
// A workgroup owns a 16 x 16 pixel tile (plus a 1-pixel halo) in LDS; each of
// its 4 wavefronts computes 4 tile rows x 64 output channels (16 MFMA tiles).
// Weights (73 KB per layer, identical for every workgroup) are read straight
// from global memory (L2-resident) as 16-byte fragments.
// The 1->64 and 64->1 layers are small and run on the vector ALUs in FP32.
#include <cmath>

#include "dg_internal.h"

namespace dg {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

static constexpr int kC = 64, kMid = 8;
static constexpr int kTile = 16, kHalo = kTile + 2;

// ------------------------------------------------------------- layouts

// FP32 master parameters, PyTorch order: w[co][ci][3][3] then b[co] per layer.
static constexpr int64_t kW0 = 0, kB0 = 576;
static constexpr int64_t kMidStride = 64 * 64 * 9 + 64;
__host__ __device__ constexpr int64_t mid_w(int l) { return 640 + (int64_t)l * kMidStride; }
__host__ __device__ constexpr int64_t mid_b(int l) { return mid_w(l) + 64 * 64 * 9; }
static constexpr int64_t kW9 = 640 + 8 * kMidStride, kB9 = kW9 + 576;
static constexpr int64_t kNParams = kB9 + 1;  // 296641

// Packed network (bytes):
//   w0f  float[64][9]           (BF16-rounded)
//   b0   float[64]
//   wm   bf16[8][9][64 co][64 ci]  (forward)
//   wmt  bf16[8][9][64 ci][64 co]  (taps flipped: backward-data)
//   bm   float[8][64]
//   w9f  float[9][64]           (BF16-rounded)
//   b9   float[1]
struct Packed {
  const float* w0;
  const float* b0;
  const bf16* wm;
  const bf16* wmt;
  const float* bm;
  const float* w9;
  const float* b9;
};
static constexpr size_t kOffW0 = 0, kOffB0 = 2304, kOffWm = 2560;
static constexpr size_t kWmBytes = (size_t)8 * 9 * 64 * 64 * 2;
static constexpr size_t kOffWmt = kOffWm + kWmBytes;
static constexpr size_t kOffBm = kOffWmt + kWmBytes;
static constexpr size_t kOffW9 = kOffBm + 8 * 64 * 4;
static constexpr size_t kOffB9 = kOffW9 + 9 * 64 * 4;
static constexpr size_t kPackedBytes = kOffB9 + 256;

__host__ __device__ inline Packed unpack(const void* base) {
  const char* c = (const char*)base;
  Packed p;
  p.w0 = (const float*)(c + kOffW0);
  p.b0 = (const float*)(c + kOffB0);
  p.wm = (const bf16*)(c + kOffWm);
  p.wmt = (const bf16*)(c + kOffWmt);
  p.bm = (const float*)(c + kOffBm);
  p.w9 = (const float*)(c + kOffW9);
  p.b9 = (const float*)(c + kOffB9);
  return p;
}

__device__ __forceinline__ float bf16_round(float v) { return (float)(bf16)v; }

__global__ void cnn_pack_kernel(const float* __restrict__ m, char* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float* w0 = (float*)(out + kOffW0);
  float* b0 = (float*)(out + kOffB0);
  bf16* wm = (bf16*)(out + kOffWm);
  bf16* wmt = (bf16*)(out + kOffWmt);
  float* bm = (float*)(out + kOffBm);
  float* w9 = (float*)(out + kOffW9);
  float* b9 = (float*)(out + kOffB9);
  if (k < 576) {  // w0[co][tap]
    w0[k] = bf16_round(m[kW0 + k]);
  }
  if (k < 64) b0[k] = m[kB0 + k];
  if (k < 8 * 9 * 64 * 64) {
    const int l = (int)(k / (9 * 64 * 64));
    const int rem = (int)(k % (9 * 64 * 64));
    const int tap = rem / 4096, a = (rem / 64) % 64, b = rem % 64;
    // forward: wm[l][tap][co=a][ci=b] = w[co][ci][tap]
    wm[k] = (bf16)m[mid_w(l) + ((int64_t)a * 64 + b) * 9 + tap];
    // backward-data: wmt[l][tap][ci=a][co=b] = w[co][ci][8 - tap]
    wmt[k] = (bf16)m[mid_w(l) + ((int64_t)b * 64 + a) * 9 + (8 - tap)];
  }
  if (k < 8 * 64) bm[k] = m[mid_b((int)(k / 64)) + k % 64];
  if (k < 576) {  // w9[tap][ci] from w9[0][ci][tap]
    const int tap = (int)(k / 64), ci = (int)(k % 64);
    w9[k] = bf16_round(m[kW9 + ci * 9 + tap]);
  }
  if (k == 0) b9[0] = m[kB9];
}

// ------------------------------------------------------------- layers

// Input layer 1 -> 64 on v_mfma_f32_16x16x4_f32 (FP32 image, BF16-rounded
// weights held as FP32, FP32 accumulation): a wavefront takes 16 pixels at a
// time; M = 16 output channels (4 blocks), N = the 16 pixels, K = 4 taps
// (3 steps cover the 9 taps, the rest zero).  Lane (l % 16, l / 16) loads
// the input of pixel l % 16 at taps l / 16, 4 + l / 16, 8 (+ zeros) and
// receives 4 channels of each block for pixel l % 16.
//   mode 0: out = relu(conv(in) + b0)
//   mode 2: also the tangent: out_t = conv(b) * (out > 0), b the Rademacher
//           probe (same MFMAs on the probe values)
__global__ void __launch_bounds__(256)
cnn_in_kernel(const float* __restrict__ in, const void* __restrict__ packed,
              bf16* __restrict__ out, bf16* __restrict__ out_t, int n, int H, int W, int mode,
              uint64_t seed, int iter) {
  const Packed P = unpack(packed);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const bool tng = mode == 2;
  // row m of block ct computes channel 32 (ct / 2) + 8 (m / 4) + 4 (ct % 2) + m % 4,
  // so that blocks 2P and 2P + 1 give a lane the 8 consecutive channels
  // 32 P + 8 (l / 16) .. + 7 of its pixel: one 16-byte store
  float wa[4][3];
  floatx4 bias[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int ch = 32 * (ct >> 1) + 8 * (lr >> 2) + 4 * (ct & 1) + (lr & 3);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int tap = 4 * s + lq;
      wa[ct][s] = tap < 9 ? P.w0[ch * 9 + tap] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[ct][j] = P.b0[32 * (ct >> 1) + 8 * lq + 4 * (ct & 1) + j];
  }
  // 32-bit index arithmetic (the host limits a call to n H W < 2^31 pixels)
  const unsigned HW = (unsigned)H * (unsigned)W, npix = (unsigned)n * HW;
  const unsigned ngroups = (npix + 15) / 16;
  for (unsigned grp = blockIdx.x * 4 + wave; grp < ngroups; grp += gridDim.x * 4) {
    const unsigned pix = grp * 16 + lr;
    const bool live = pix < npix;
    const unsigned img = live ? pix / HW : 0;
    const int rem = live ? (int)(pix - img * HW) : 0;
    const int y = rem / W, x = rem - y * W;
    float v[3], pb[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int tap = 4 * s + lq;
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      const bool ok = live && tap < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W;
      v[s] = ok ? in[(int64_t)img * HW + yy * W + xx] : 0.0f;
      pb[s] = 0.0f;
      if (tng && ok) pb[s] = probe_sign(seed, iter, (uint64_t)((int64_t)yy * W + xx));
    }
#pragma unroll
    for (int P2 = 0; P2 < 2; ++P2) {
      bf16x8 o8, t8;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int ct = 2 * P2 + b;
        floatx4 cf = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 3; ++s)
          cf = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[ct][s], v[s], cf, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) o8[4 * b + j] = (bf16)fmaxf(cf[j] + bias[ct][j], 0.0f);
        if (tng) {
          floatx4 tf = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int s = 0; s < 3; ++s)
            tf = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[ct][s], pb[s], tf, 0, 0, 0);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            t8[4 * b + j] = (bf16)(((float)o8[4 * b + j] > 0.0f) ? tf[j] : 0.0f);
        }
      }
      // this lane's output column is pixel grp * 16 + lr (= pix)
      if (live) {
        *(bf16x8*)(out + (int64_t)pix * kC + 32 * P2 + 8 * lq) = o8;
        if (tng) *(bf16x8*)(out_t + (int64_t)pix * kC + 32 * P2 + 8 * lq) = t8;
      }
    }
  }
}

static unsigned int in_grid(int64_t npix) {
  const int64_t g = (npix + 63) / 64;  // four 16-pixel groups per workgroup
  return (unsigned int)(g < 4096 ? g : 4096);
}

// 64 -> 64 layer on MFMA.
//   mode 0: out = relu(conv(in, Wl) + bl)
//   mode 1: out = conv(in, Wl) * (mask > 0)
// W: bf16[9][64 out][64 in].
//
// One 512-thread workgroup per compute unit (two wavefronts per SIMD) walks
// output tiles of kMidTH x kMidTW pixels.  The layer's weights (72 KiB) are
// staged in LDS once per workgroup; each tile's input halo ((kMidTH+2) x
// (kMidTW+2) pixels x 64 channels, 76.5 KiB) is staged per tile, all of a
// thread's loads in flight at once.  Both LDS arrays store 16-byte channel
// chunks XOR-swizzled by the row index (chunk c of row p at c ^ (p & 7)), so
// the lanes that read one fragment row hit distinct 16-byte bank groups.
// Wavefront w computes tile rows 4w .. 4w+3 for all 64 output channels with
// v_mfma_f32_16x16x32_bf16: per K-step (tap, 32-channel half) 4 weight
// fragments and 4 pixel fragments feed 16 MFMAs; the compiler shares the
// pixel fragments of a row between the three taps of one column.  (The
// 32 x 32 x 16 form has a higher peak, but in this tiling it moves more LDS
// bytes per MFMA and measured slower.)
static constexpr int kMidThreads = 512, kMidWaves = kMidThreads / 64;
static constexpr int kMidTH = 32, kMidTW = 16;
static constexpr int kMidHH = kMidTH + 2, kMidHW = kMidTW + 2;
static constexpr int kMidRows = kMidTH / kMidWaves;  // tile rows per wavefront
static constexpr int kHaloChunks = kMidHH * kMidHW * 8;
static constexpr int kHaloRounds = (kHaloChunks + kMidThreads - 1) / kMidThreads;

__device__ __forceinline__ int swz(int row, int chunk) { return (row << 3) + (chunk ^ (row & 7)); }

// Output-channel order of the MFMA blocks: row m of block ct (LDS weight row
// 16 ct + m of a tap) computes channel 32 (ct / 2) + 8 (m / 4) + 4 (ct % 2)
// + m % 4, so blocks 2P and 2P + 1 give a lane (l % 16, l / 16) the 8
// consecutive channels 32 P + 8 (l / 16) .. + 7 of its pixel (one 16-byte
// store).  w_row maps a packed weight row (tap, channel) to its LDS row.
__device__ __forceinline__ int w_row(int row) {
  const int tap = row >> 6, co = row & 63;
  return tap * 64 + (2 * (co >> 5) + ((co >> 2) & 1)) * 16 + 4 * ((co >> 3) & 3) + (co & 3);
}

__host__ __device__ inline int mid_tiles(int n, int H, int W) {
  return n * ((H + kMidTH - 1) / kMidTH) * ((W + kMidTW - 1) / kMidTW);
}

// Load one tile's halo into registers (zero outside the image); interior
// tiles skip the per-chunk bounds tests.
__device__ __forceinline__ void halo_fetch(const bf16* __restrict__ in, int tile, int tiles_x,
                                           int tiles_y, int H, int W, bf16x8 (&hr)[kHaloRounds]) {
  const int img = tile / (tiles_x * tiles_y);
  const int trem = tile % (tiles_x * tiles_y);
  const int y0 = (trem / tiles_x) * kMidTH - 1, x0 = (trem % tiles_x) * kMidTW - 1;
  const bf16* base = in + ((int64_t)img * H * W + (int64_t)y0 * W + x0) * kC;
  const bool interior = y0 >= 0 && x0 >= 0 && y0 + kMidHH <= H && x0 + kMidHW <= W;
#pragma unroll
  for (int q = 0; q < kHaloRounds; ++q) {
    const int e = q * kMidThreads + threadIdx.x;
    const int pix = e >> 3, ch = e & 7;
    const int hy = pix / kMidHW, hx = pix - hy * kMidHW;
#pragma unroll
    for (int j = 0; j < 8; ++j) hr[q][j] = (bf16)0.0f;
    const bool inb = (q + 1 < kHaloRounds || e < kHaloChunks) &&
                     (interior || ((unsigned)(y0 + hy) < (unsigned)H && (unsigned)(x0 + hx) < (unsigned)W));
    if (inb) hr[q] = *(const bf16x8*)(base + ((int64_t)hy * W + hx) * kC + ch * 8);
  }
}

__device__ __forceinline__ void halo_store(bf16x8* sX, const bf16x8 (&hr)[kHaloRounds]) {
#pragma unroll
  for (int q = 0; q < kHaloRounds; ++q) {
    const int e = q * kMidThreads + threadIdx.x;
    if (e < kHaloChunks) sX[swz(e >> 3, e & 7)] = hr[q];
  }
}

template <int MODE>
__global__ void __launch_bounds__(kMidThreads)
cnn_mid_kernel(const bf16* __restrict__ in, const bf16* __restrict__ Wt,
               const float* __restrict__ bias, const bf16* __restrict__ mask,
               bf16* __restrict__ out, int n, int H, int W) {
  __shared__ bf16x8 sW[9 * 64 * 8];            // [tap][co] rows of 8 chunks
  __shared__ bf16x8 sX[kMidHH * kMidHW * 8];   // [halo pixel] rows of 8 chunks
  __shared__ floatx4 sB[16];                   // biases (mode 0)
  const int tiles_x = (W + kMidTW - 1) / kMidTW, tiles_y = (H + kMidTH - 1) / kMidTH;
  const int ntiles = n * tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;  // fragment row (pixel / co) and k chunk
  bf16x8 hr[kHaloRounds];
  int tile = blockIdx.x;
  {
    // weights and the first halo: every load is issued before the first LDS
    // store, so the staging costs one memory latency
    constexpr int kRounds = 9 * 64 * 8 / kMidThreads;
    bf16x8 wr[kRounds];
#pragma unroll
    for (int q = 0; q < kRounds; ++q)
      wr[q] = *(const bf16x8*)(Wt + (int64_t)(q * kMidThreads + threadIdx.x) * 8);
    if (tile < ntiles) halo_fetch(in, tile, tiles_x, tiles_y, H, W, hr);
    if (MODE == 0 && threadIdx.x < 16)
      sB[threadIdx.x] = floatx4{bias[threadIdx.x * 4], bias[threadIdx.x * 4 + 1],
                                bias[threadIdx.x * 4 + 2], bias[threadIdx.x * 4 + 3]};
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      const int e = q * kMidThreads + threadIdx.x;
      sW[swz(w_row(e >> 3), e & 7)] = wr[q];
    }
  }
  if (tile < ntiles) halo_store(sX, hr);
  __syncthreads();
  for (; tile < ntiles; tile += gridDim.x) {
    const int img = tile / (tiles_x * tiles_y);
    const int trem = tile % (tiles_x * tiles_y);
    const int y0 = (trem / tiles_x) * kMidTH, x0 = (trem % tiles_x) * kMidTW;
    const int64_t ibase = (int64_t)img * H * W;
    const int next = tile + gridDim.x;
    floatx4 acc[kMidRows][4];
#pragma unroll
    for (int a = 0; a < kMidRows; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ty = tap / 3, tx = tap % 3;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int chunk = half * 4 + lq;
        bf16x8 af[4], bfr[kMidRows];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) af[ct] = sW[swz(tap * 64 + ct * 16 + lr, chunk)];
#pragma unroll
        for (int rr = 0; rr < kMidRows; ++rr)
          bfr[rr] = sX[swz((wave * kMidRows + rr + ty) * kMidHW + lr + tx, chunk)];
#pragma unroll
        for (int rr = 0; rr < kMidRows; ++rr)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
            acc[rr][ct] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ct], bfr[rr], acc[rr][ct], 0, 0, 0);
      }
    }
    // C layout: lane holds pixel column lr; blocks 2P, 2P + 1 hold its
    // channels 32 P + 8 lq .. + 7 (see w_row)
    bf16x8 m8[kMidRows][2];
    if (MODE != 0) {
#pragma unroll
      for (int rr = 0; rr < kMidRows; ++rr) {
        const int yy = y0 + wave * kMidRows + rr, xx = x0 + lr;
        const bool ok = yy < H && xx < W;
        const int64_t pbase = (ibase + (int64_t)(ok ? yy : 0) * W + (ok ? xx : 0)) * kC;
#pragma unroll
        for (int P2 = 0; P2 < 2; ++P2)
          m8[rr][P2] = *(const bf16x8*)(mask + pbase + 32 * P2 + 8 * lq);
      }
    }
#pragma unroll
    for (int rr = 0; rr < kMidRows; ++rr) {
      const int yy = y0 + wave * kMidRows + rr, xx = x0 + lr;
      if (yy >= H || xx >= W) continue;
      const int64_t pbase = (ibase + (int64_t)yy * W + xx) * kC;
#pragma unroll
      for (int P2 = 0; P2 < 2; ++P2) {
        bf16x8 o8;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int ct = 2 * P2 + b;
          const floatx4 b4 = (MODE == 0) ? sB[8 * P2 + 2 * lq + b] : floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (MODE == 0)
              o8[4 * b + j] = (bf16)fmaxf(acc[rr][ct][j] + b4[j], 0.0f);
            else
              o8[4 * b + j] = (bf16)(((float)m8[rr][P2][4 * b + j] > 0.0f) ? acc[rr][ct][j] : 0.0f);
          }
        }
        *(bf16x8*)(out + pbase + 32 * P2 + 8 * lq) = o8;
      }
    }
    if (next < ntiles) {
      halo_fetch(in, next, tiles_x, tiles_y, H, W, hr);
      __syncthreads();  // every wavefront is done reading this tile's halo
      halo_store(sX, hr);
      __syncthreads();
    }
  }
}

// One workgroup per compute unit (the kernel's LDS use admits no second),
// never more workgroups than tiles.
static unsigned int mid_grid(int n, int H, int W) {
  const int t = mid_tiles(n, H, W);
  return (unsigned int)(t < 256 ? t : 256);
}

// The forward layer and its tangent in one pass (denoiser inference):
//   out  = relu(conv(in, Wl) + bl)
//   outt = conv(int, Wl) * (out > 0)
// Same K order and MFMA as cnn_mid_kernel, so both outputs are bitwise those
// of the two separate passes; the tangent's ReLU pattern comes from the
// forward result in registers instead of a reread of the stored activation,
// and every weight fragment read from LDS feeds both images.  Tiles are
// 16 x 16 (two halos of 18 x 18 pixels x 64 channels next to the 72 KiB of
// weights); wavefront w computes tile rows 2w, 2w + 1 of both images.
static constexpr int kDualT = 16, kDualH = kDualT + 2;
static constexpr int kDualRows = kDualT / kMidWaves;                // 2
static constexpr int kDualChunks = kDualH * kDualH * 8;            // per image
static constexpr int kDualRounds = (2 * kDualChunks + kMidThreads - 1) / kMidThreads;
static constexpr int kDualEarly = 6;

__host__ __device__ inline int dual_tiles(int n, int H, int W) {
  return n * ((H + kDualT - 1) / kDualT) * ((W + kDualT - 1) / kDualT);
}

// Rounds Q0 <= q < Q1 of a tile's halo loads into hr.
template <int Q0 = 0, int Q1 = kDualRounds>
__device__ __forceinline__ void dual_fetch(const bf16* __restrict__ in0, const bf16* __restrict__ in1,
                                           int tile, int tiles_x, int tiles_y, int H, int W,
                                           bf16x8 (&hr)[kDualRounds]) {
  const int img = tile / (tiles_x * tiles_y);
  const int trem = tile % (tiles_x * tiles_y);
  const int y0 = (trem / tiles_x) * kDualT - 1, x0 = (trem % tiles_x) * kDualT - 1;
  const int64_t off = ((int64_t)img * H * W + (int64_t)y0 * W + x0) * kC;
  const bool interior = y0 >= 0 && x0 >= 0 && y0 + kDualH <= H && x0 + kDualH <= W;
#pragma unroll
  for (int q = Q0; q < Q1; ++q) {
    const int e = q * kMidThreads + threadIdx.x;
    const int which = e >= kDualChunks;
    const int e2 = e - which * kDualChunks;
    const int pix = e2 >> 3, ch = e2 & 7;
    const int hy = pix / kDualH, hx = pix - hy * kDualH;
#pragma unroll
    for (int j = 0; j < 8; ++j) hr[q][j] = (bf16)0.0f;
    const bool inb = e < 2 * kDualChunks &&
                     (interior || ((unsigned)(y0 + hy) < (unsigned)H && (unsigned)(x0 + hx) < (unsigned)W));
    if (inb) hr[q] = *(const bf16x8*)((which ? in1 : in0) + off + ((int64_t)hy * W + hx) * kC + ch * 8);
  }
}

__device__ __forceinline__ void dual_store(bf16x8* sX, const bf16x8 (&hr)[kDualRounds]) {
#pragma unroll
  for (int q = 0; q < kDualRounds; ++q) {
    const int e = q * kMidThreads + threadIdx.x;
    const int which = e >= kDualChunks;
    const int e2 = e - which * kDualChunks;
    if (e < 2 * kDualChunks) sX[which * kDualChunks + swz(e2 >> 3, e2 & 7)] = hr[q];
  }
}

__global__ void __launch_bounds__(kMidThreads)
cnn_mid_dual_kernel(const bf16* __restrict__ in, const bf16* __restrict__ int_,
                    const bf16* __restrict__ Wt, const float* __restrict__ bias,
                    bf16* __restrict__ out, bf16* __restrict__ outt, int n, int H, int W) {
  __shared__ bf16x8 sW[9 * 64 * 8];          // [tap][co] rows of 8 chunks
  __shared__ bf16x8 sX[2 * kDualChunks];     // two halos, [image][pixel] rows of 8 chunks
  __shared__ floatx4 sB[16];
  const int tiles_x = (W + kDualT - 1) / kDualT, tiles_y = (H + kDualT - 1) / kDualT;
  const int ntiles = n * tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  bf16x8 hr[kDualRounds];
  int tile = blockIdx.x;
  {
    constexpr int kRounds = 9 * 64 * 8 / kMidThreads;
    bf16x8 wr[kRounds];
#pragma unroll
    for (int q = 0; q < kRounds; ++q)
      wr[q] = *(const bf16x8*)(Wt + (int64_t)(q * kMidThreads + threadIdx.x) * 8);
    if (tile < ntiles) dual_fetch(in, int_, tile, tiles_x, tiles_y, H, W, hr);
    if (threadIdx.x < 16)
      sB[threadIdx.x] = floatx4{bias[threadIdx.x * 4], bias[threadIdx.x * 4 + 1],
                                bias[threadIdx.x * 4 + 2], bias[threadIdx.x * 4 + 3]};
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      const int e = q * kMidThreads + threadIdx.x;
      sW[swz(w_row(e >> 3), e & 7)] = wr[q];
    }
  }
  if (tile < ntiles) dual_store(sX, hr);
  __syncthreads();
  for (; tile < ntiles; tile += gridDim.x) {
    const int img = tile / (tiles_x * tiles_y);
    const int trem = tile % (tiles_x * tiles_y);
    const int y0 = (trem / tiles_x) * kDualT, x0 = (trem % tiles_x) * kDualT;
    const int64_t ibase = (int64_t)img * H * W;
    const int next = tile + gridDim.x;
    // the first kDualEarly rounds of the next tile's halo loads are issued
    // now and stay in flight while this tile's MFMAs run (all of them would
    // not fit the register budget beside the accumulators)
    if (next < ntiles) dual_fetch<0, kDualEarly>(in, int_, next, tiles_x, tiles_y, H, W, hr);
    floatx4 acc[2][kDualRows][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int a = 0; a < kDualRows; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[m][a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ty = tap / 3, tx = tap % 3;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int chunk = half * 4 + lq;
        bf16x8 af[4], bfr[2][kDualRows];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) af[ct] = sW[swz(tap * 64 + ct * 16 + lr, chunk)];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int rr = 0; rr < kDualRows; ++rr)
            bfr[m][rr] = sX[m * kDualChunks +
                            swz((wave * kDualRows + rr + ty) * kDualH + lr + tx, chunk)];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int rr = 0; rr < kDualRows; ++rr)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
              acc[m][rr][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ct], bfr[m][rr],
                                                                       acc[m][rr][ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int rr = 0; rr < kDualRows; ++rr) {
      const int yy = y0 + wave * kDualRows + rr, xx = x0 + lr;
      if (yy >= H || xx >= W) continue;
      const int64_t pbase = (ibase + (int64_t)yy * W + xx) * kC;
#pragma unroll
      for (int P2 = 0; P2 < 2; ++P2) {
        bf16x8 o8, t8;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int ct = 2 * P2 + b;
          const floatx4 b4 = sB[8 * P2 + 2 * lq + b];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            o8[4 * b + j] = (bf16)fmaxf(acc[0][rr][ct][j] + b4[j], 0.0f);
            t8[4 * b + j] = (bf16)(((float)o8[4 * b + j] > 0.0f) ? acc[1][rr][ct][j] : 0.0f);
          }
        }
        *(bf16x8*)(out + pbase + 32 * P2 + 8 * lq) = o8;
        *(bf16x8*)(outt + pbase + 32 * P2 + 8 * lq) = t8;
      }
    }
    if (next < ntiles) {
      dual_fetch<kDualEarly, kDualRounds>(in, int_, next, tiles_x, tiles_y, H, W, hr);
      __syncthreads();  // every wavefront is done reading this tile's halos
      dual_store(sX, hr);
      __syncthreads();
    }
  }
}

static unsigned int dual_grid(int n, int H, int W) {
  const int t = dual_tiles(n, H, W);
  return (unsigned int)(t < 256 ? t : 256);
}

// Output layer 64 -> 1, 16 x 16 output tiles (grid stride).  Pass 1: for
// every pixel q of the 18 x 18 halo, the 9 tap dot products
// d_t(q) = act[q] . w9[t] on v_mfma_f32_16x16x32_bf16 (M = 16 tap rows of
// which 9 are used, N = 16 halo pixels, K = 2 x 32 channels; the B fragment
// of a lane is one 16-byte channel chunk of one pixel, as stored), into LDS;
// pass 2: f(p) = b9 + sum_t d_t(p + off_t).  All halo loads of a tile are
// issued before the first is used.
//   mode 0 (primal):   out = r - (conv(act) + b9)
//   mode 2 (training): f = conv(act) + b9; res = r - f - clean;
//                      out = g_f = -2 res / count; loss partial per block
//   mode 3 (denoiser with its tangent): out = r - (conv(act) + b9) and
//                      out2 = out + eps (b - conv(actt)), so that
//                      b^T (out2 - out) / (N eps) = b^T J_D b / N
static constexpr int kOutT = 16, kOutH = kOutT + 2;
static constexpr int kOutGroups = (kOutH * kOutH + 15) / 16;  // 16-pixel groups per halo
static constexpr int kOutPerWave = (2 * kOutGroups + 3) / 4;   // both images, 4 wavefronts

__host__ __device__ inline int out_tiles(int n, int H, int W) {
  return n * ((H + kOutT - 1) / kOutT) * ((W + kOutT - 1) / kOutT);
}

__global__ void __launch_bounds__(256)
cnn_out_kernel(const bf16* __restrict__ act, const bf16* __restrict__ actt,
               const void* __restrict__ packed, const float* __restrict__ r,
               const float* __restrict__ clean, float* __restrict__ out, float* __restrict__ out2,
               int n, int H, int W, int mode, const double* __restrict__ eps_ptr, int eps_stride,
               uint64_t seed, int iter, double* __restrict__ loss_partials, double inv_count) {
  __shared__ float sd[2][kOutH * kOutH][9];
  __shared__ double red[4];
  const Packed P = unpack(packed);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  bf16x8 wa[2];  // A fragments: tap lr (zero beyond 8), channel chunks lq and 4 + lq
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      wa[h][j] = (bf16)(lr < 9 ? P.w9[lr * 64 + (h * 4 + lq) * 8 + j] : 0.0f);
  const int ntask = (mode == 3 ? 2 : 1) * kOutGroups;
  const int tiles_x = (W + kOutT - 1) / kOutT, tiles_y = (H + kOutT - 1) / kOutT;
  const int ntiles = n * tiles_x * tiles_y;
  const int64_t HW = (int64_t)H * W;
  double lsum = 0.0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int img = tile / (tiles_x * tiles_y);
    const int trem = tile % (tiles_x * tiles_y);
    const int y0 = (trem / tiles_x) * kOutT, x0 = (trem % tiles_x) * kOutT;
    const int64_t ibase = (int64_t)img * HW;
    bf16x8 hv[kOutPerWave][2];
#pragma unroll
    for (int k = 0; k < kOutPerWave; ++k) {
      const int task = wave + 4 * k;
      const int which = task >= kOutGroups;
      const int q = (task - which * kOutGroups) * 16 + lr;
      const int yy = y0 - 1 + q / kOutH, xx = x0 - 1 + q % kOutH;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 8; ++j) hv[k][h][j] = (bf16)0.0f;
      if (task < ntask && q < kOutH * kOutH && yy >= 0 && yy < H && xx >= 0 && xx < W) {
        const bf16* src = (which ? actt : act) + (ibase + (int64_t)yy * W + xx) * kC;
        hv[k][0] = *(const bf16x8*)(src + lq * 8);
        hv[k][1] = *(const bf16x8*)(src + (4 + lq) * 8);
      }
    }
    __syncthreads();  // the previous tile's pass 2 is done with sd
#pragma unroll
    for (int k = 0; k < kOutPerWave; ++k) {
      const int task = wave + 4 * k;
      if (task >= ntask) break;  // wavefront-uniform
      const int which = task >= kOutGroups;
      const int q = (task - which * kOutGroups) * 16 + lr;
      floatx4 d = {0.0f, 0.0f, 0.0f, 0.0f};
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[0], hv[k][0], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[1], hv[k][1], d, 0, 0, 0);
      // this lane holds taps 4 lq .. 4 lq + 3 of halo pixel q
      if (q < kOutH * kOutH) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * lq + j < 9) sd[which][q][4 * lq + j] = d[j];
      }
    }
    __syncthreads();
    const int ty = threadIdx.x / kOutT, tx = threadIdx.x % kOutT;
    const int y = y0 + ty, x = x0 + tx;
    if (y < H && x < W) {
      float f = P.b9[0];
#pragma unroll
      for (int t = 0; t < 9; ++t) f += sd[0][(ty + t / 3) * kOutH + tx + t % 3][t];
      const int64_t rem = (int64_t)y * W + x, pix = ibase + rem;
      if (mode == 2) {
        const float res = r[pix] - f - clean[pix];
        lsum += (double)res * (double)res;
        out[pix] = (float)(-2.0 * (double)res * inv_count);
      } else {
        const float d0 = r[pix] - f;
        out[pix] = d0;
        if (mode == 3) {
          float g = 0.0f;
#pragma unroll
          for (int t = 0; t < 9; ++t) g += sd[1][(ty + t / 3) * kOutH + tx + t % 3][t];
          const float b = probe_sign(seed, iter, (uint64_t)rem);
          out2[pix] = __fmaf_rn((float)eps_ptr[(int64_t)img * eps_stride], b - g, d0);
        }
      }
    }
  }
  if (mode == 2) {
    const double bs = block_sum(lsum, red);
    if (threadIdx.x == 0) loss_partials[blockIdx.x] = bs;
  }
}

// Workgroups of the output layer (loss partials in mode 2: one per workgroup).
static unsigned int out_grid(int n, int H, int W) {
  const int t = out_tiles(n, H, W);
  return (unsigned int)(t < 2048 ? t : 2048);
}

// ------------------------------------------------------------- backward

// g8[p][ci] = (sum_tap g_f[p - tap + 1] w9[tap][ci]) * (act8[p][ci] > 0)
__global__ void __launch_bounds__(256)
cnn_out_bwd_kernel(const float* __restrict__ gf, const void* __restrict__ packed,
                   const bf16* __restrict__ act, bf16* __restrict__ g8, int n, int H, int W) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)n * H * W;
  if (pix >= npix) return;
  const Packed P = unpack(packed);
  const int img = (int)(pix / ((int64_t)H * W));
  const int rem = (int)(pix % ((int64_t)H * W));
  const int y = rem / W, x = rem % W;
  float g[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    // output pixel (y - ty + 1, x - tx + 1) reads this pixel through tap t
    const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
    g[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
               ? gf[(int64_t)img * H * W + (int64_t)yy * W + xx] : 0.0f;
  }
  const bf16* a = act + pix * kC;
  bf16* o = g8 + pix * kC;
  for (int c0 = 0; c0 < kC; c0 += 8) {
    const bf16x8 av = *(const bf16x8*)(a + c0);
    bf16x8 pack;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float s = 0.0f;
#pragma unroll
      for (int t = 0; t < 9; ++t) s = __fmaf_rn(P.w9[t * 64 + c0 + j], g[t], s);
      pack[j] = (bf16)(((float)av[j] > 0.0f) ? s : 0.0f);
    }
    *(bf16x8*)(o + c0) = pack;
  }
}

// Weight gradient of a 64 -> 64 layer: dW[tap][co][ci] += sum_p g[p][co] in[p + tap - 1][ci]
// (and db[co] += sum_p g[p][co]).  Each workgroup walks tiles with stride
// gridDim.x and accumulates in registers; its partial goes to
// part[blockIdx][9*64*64 + 64], summed by cnn_reduce_kernel.
// MFMA: A = g^T (16 co x 32 pixels), B = in (32 pixels x 16 ci); the tiles
// are staged channel-major in LDS so that 8 consecutive pixels of one
// channel are contiguous.
static constexpr int kGTP = kTile * kTile + 8;       // g^T row pitch (pixels)
static constexpr int kITP = kHalo * kHalo + 8;       // in^T row pitch
__global__ void __launch_bounds__(256)
cnn_wgrad_kernel(const bf16* __restrict__ g, const bf16* __restrict__ in, float* __restrict__ part,
                 int n, int H, int W) {
  __shared__ __attribute__((aligned(16))) bf16 sG[kC * kGTP];
  __shared__ __attribute__((aligned(16))) bf16 sI[kC * kITP];
  const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
  const int ntiles = n * tiles_x * tiles_y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;  // wave = co tile
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  floatx4 acc[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[t][c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  float dbias = 0.0f;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int img = tile / (tiles_x * tiles_y);
    const int trem = tile % (tiles_x * tiles_y);
    const int y0 = (trem / tiles_x) * kTile, x0 = (trem % tiles_x) * kTile;
    const int64_t ibase = (int64_t)img * H * W;
    __syncthreads();
    for (int e = threadIdx.x; e < kTile * kTile * 8; e += blockDim.x) {
      const int pix = e >> 3, ch = (e & 7) * 8;
      const int yy = y0 + pix / kTile, xx = x0 + pix % kTile;
      bf16x8 v;
      if (yy < H && xx < W)
        v = *(const bf16x8*)(g + (ibase + (int64_t)yy * W + xx) * kC + ch);
      else
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (bf16)0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j) sG[(ch + j) * kGTP + pix] = v[j];
    }
    for (int e = threadIdx.x; e < kHalo * kHalo * 8; e += blockDim.x) {
      const int pix = e >> 3, ch = (e & 7) * 8;
      const int yy = y0 - 1 + pix / kHalo, xx = x0 - 1 + pix % kHalo;
      bf16x8 v;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = *(const bf16x8*)(in + (ibase + (int64_t)yy * W + xx) * kC + ch);
      else
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (bf16)0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j) sI[(ch + j) * kITP + pix] = v[j];
    }
    __syncthreads();
    // bias gradient of this wave's 16 channels: lanes 0..15 sum their channel
    if (lane < 16) {
      const bf16* row = sG + (wave * 16 + lane) * kGTP;
      for (int p = 0; p < kTile * kTile; ++p) dbias += (float)row[p];
    }
    // K = 256 tile pixels in 8 steps of 32 (two tile rows per step)
    for (int ks = 0; ks < 8; ++ks) {
      const int p0 = ks * 32 + lk;  // 8 consecutive pixels of one tile row
      const bf16x8 a = *(const bf16x8*)(sG + (wave * 16 + lr) * kGTP + p0);
      const int py = p0 / kTile, px = p0 % kTile;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int hy = py + tap / 3, hx = px + tap % 3;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16* src = sI + (c * 16 + lr) * kITP + hy * kHalo + hx;
          bf16x8 b;
#pragma unroll
          for (int j = 0; j < 8; ++j) b[j] = src[j];
          acc[tap][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tap][c], 0, 0, 0);
        }
      }
    }
  }
  // C layout: lane holds ci column lr, co rows 4*(lane>>4)+j of this wave's co tile
  float* dst = part + (int64_t)blockIdx.x * (9 * 64 * 64 + 64);
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = wave * 16 + (lane >> 4) * 4 + j, ci = c * 16 + lr;
        dst[(tap * 64 + co) * 64 + ci] = acc[tap][c][j];
      }
  if (lane < 16) dst[9 * 64 * 64 + wave * 16 + lane] = dbias;
}

// Small layers' weight gradients (FP32 vector), per-block partials.
//   which 0: dW0[co][tap] = sum_p g0[p][co] r[p + tap - 1], db0[co] = sum_p g0[p][co]
//   which 9: dW9[ci][tap] = sum_p gf[p] act8[p + tap - 1][ci], db9 = sum_p gf[p]
// part row: 576 + 64 floats (which 0) or 576 + 1 (which 9).
__global__ void __launch_bounds__(256)
cnn_small_wgrad_kernel(const bf16* __restrict__ gact, const float* __restrict__ img_in,
                       const float* __restrict__ gf, const bf16* __restrict__ act8,
                       float* __restrict__ part, int n, int H, int W, int which) {
  __shared__ float red[256];
  const int64_t npix = (int64_t)n * H * W;
  // thread handles one (channel, tap) slot for a strided set of pixels:
  // 64 channels x 9 taps = 576 slots + bias slots, blockDim 256 -> loop
  float* dst = part + (int64_t)blockIdx.x * 640;
  for (int slot = threadIdx.x; slot < 640; slot += blockDim.x) {
    float s = 0.0f;
    const bool is_w = slot < 576;
    const int ch = is_w ? slot / 9 : slot - 576;
    const int tap = is_w ? slot % 9 : 0;
    if (which == 9 && !is_w && ch > 0) {
      dst[slot] = 0.0f;
      continue;
    }
    for (int64_t p = blockIdx.x; p < npix; p += gridDim.x) {
      const int im = (int)(p / ((int64_t)H * W));
      const int rem = (int)(p % ((int64_t)H * W));
      const int y = rem / W, x = rem % W;
      if (which == 0) {
        const float gv = (float)gact[p * kC + ch];
        if (!is_w) {
          s += gv;
        } else {
          const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            s = __fmaf_rn(gv, img_in[(int64_t)im * H * W + (int64_t)yy * W + xx], s);
        }
      } else {
        const float gv = gf[p];
        if (!is_w) {
          s += gv;
        } else {
          const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            s = __fmaf_rn(gv, (float)act8[((int64_t)im * H * W + (int64_t)yy * W + xx) * kC + ch], s);
        }
      }
    }
    dst[slot] = s;
  }
  (void)red;
}

// Sum `nrows` partial rows of length `len` into `out` (fixed order).
__global__ void cnn_reduce_kernel(const float* __restrict__ part, int nrows, int len,
                                  float* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  float s = 0.0f;
  for (int r = 0; r < nrows; ++r) s += part[(int64_t)r * len + k];
  out[k] = s;
}

// Scatter reduced gradients into the master layout.
//   mid: red[(tap*64 + co)*64 + ci] -> grad[mid_w(l) + (co*64 + ci)*9 + tap], bias after 9*64*64
__global__ void cnn_scatter_mid(const float* __restrict__ red, float* __restrict__ grad, int l) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 9 * 64 * 64) {
    const int tap = k / 4096, co = (k / 64) % 64, ci = k % 64;
    grad[mid_w(l) + ((int64_t)co * 64 + ci) * 9 + tap] = red[k];
  } else if (k < 9 * 64 * 64 + 64) {
    grad[mid_b(l) + (k - 9 * 64 * 64)] = red[k];
  }
}

__global__ void cnn_scatter_small(const float* __restrict__ red, float* __restrict__ grad,
                                  int which) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (which == 0) {
    if (k < 576) grad[kW0 + k] = red[k];  // [co][tap] == master [co][0][ty][tx]
    else if (k < 640) grad[kB0 + (k - 576)] = red[k];
  } else {
    if (k < 576) grad[kW9 + k] = red[k];  // [ci][tap] == master [0][ci][ty][tx]
    else if (k == 576) grad[kB9] = red[k];
  }
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters.
__global__ void cnn_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                float b1, float b2, float eps, float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void cnn_loss_finish(const double* __restrict__ partials, int n, double scale,
                                double* __restrict__ out) {
  __shared__ double red[4];
  const double t = finish_sum(partials, n, red);
  if (threadIdx.x == 0) *out = t * scale;
}

// ------------------------------------------------------------- host side

struct CnnWork {
  bf16* act[9];   // post-ReLU activations of the 9 hidden layers
  bf16* tan[2];   // tangent / gradient ping-pong
  float* f;       // output-layer buffer (training: g_f)
  float* part;    // gradient partials
  float* red;     // reduced gradient
  double* dpart;  // loss partials
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
static constexpr int kWgradBlocks = 128;

static size_t cnn_work_layout(int64_t npix, void* base, CnnWork* w) {
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = c ? c + off : nullptr;
    off += a256(b);
    return p;
  };
  CnnWork t;
  const size_t ab = (size_t)npix * kC * sizeof(bf16);
  for (int l = 0; l < 9; ++l) t.act[l] = (bf16*)take(ab);
  t.tan[0] = (bf16*)take(ab);
  t.tan[1] = (bf16*)take(ab);
  t.f = (float*)take(sizeof(float) * (size_t)npix);
  t.part = (float*)take(sizeof(float) * (size_t)kWgradBlocks * (9 * 64 * 64 + 64));
  t.red = (float*)take(sizeof(float) * (9 * 64 * 64 + 64));
  t.dpart = (double*)take(sizeof(double) * 65536);
  if (w) *w = t;
  return off;
}

size_t cnn_work_bytes(int64_t npix) { return cnn_work_layout(npix, nullptr, nullptr); }

static unsigned int g256(int64_t n) { return (unsigned int)((n + 255) / 256); }

// Forward pass storing activations; out = r - f(r) when out != null.
static dg_status cnn_forward(const void* packed, const float* r, float* out, int n, int H, int W,
                             CnnWork& w, hipStream_t st) {
  const Packed P = unpack(packed);
  const int64_t npix = (int64_t)n * H * W;
  DG_ARG_CHECK(npix < ((int64_t)1 << 31), "CNN: at most 2^31 - 1 pixels per call");
  hipLaunchKernelGGL(cnn_in_kernel, dim3(in_grid(npix)), dim3(256), 0, st, r, packed,
                     w.act[0], (bf16*)nullptr, n, H, W, 0, (uint64_t)0, 0);
  DG_LAUNCH_CHECK("cnn_in_kernel");
  const unsigned int tiles = mid_grid(n, H, W);
  for (int l = 0; l < kMid; ++l) {
    hipLaunchKernelGGL(cnn_mid_kernel<0>, dim3(tiles), dim3(kMidThreads), 0, st, w.act[l],
                       P.wm + (size_t)l * 9 * 64 * 64, P.bm + l * 64, (const bf16*)nullptr,
                       w.act[l + 1], n, H, W);
    DG_LAUNCH_CHECK("cnn_mid_kernel");
  }
  if (out) {
    hipLaunchKernelGGL(cnn_out_kernel, dim3(out_grid(n, H, W)), dim3(256), 0, st, w.act[8],
                       (const bf16*)nullptr, packed, r, (const float*)nullptr, out, (float*)nullptr,
                       n, H, W, 0, (const double*)nullptr, 0, (uint64_t)0, 0, (double*)nullptr, 0.0);
    DG_LAUNCH_CHECK("cnn_out_kernel");
  }
  return DG_OK;
}

dg_status cnn_check_params(const dg_plan* p, const void* params) {
  DG_ARG_CHECK(params != nullptr, "denoise: CNN params must not be NULL");
  const dg_cnn_params* cp = (const dg_cnn_params*)params;
  DG_ARG_CHECK(cp->weights != nullptr, "denoise: CNN weights must not be NULL");
  DG_ARG_CHECK(cp->work != nullptr, "denoise: CNN work buffer must not be NULL");
  (void)p;
  return DG_OK;
}

// Denoiser and tangent together: x_den = r - f(r) and x_pert = x_den +
// eps (b - J_f b) with every layer's forward and tangent in one launch.
static dg_status cnn_denoise_dual(const void* packed, const float* r, float* xden, float* xpert,
                                  const double* eps, int eps_stride, uint64_t seed, int iter, int n,
                                  int H, int W, CnnWork& w, hipStream_t st) {
  const Packed P = unpack(packed);
  const int64_t npix = (int64_t)n * H * W;
  DG_ARG_CHECK(npix < ((int64_t)1 << 31), "CNN: at most 2^31 - 1 pixels per call");
  hipLaunchKernelGGL(cnn_in_kernel, dim3(in_grid(npix)), dim3(256), 0, st, r, packed, w.act[0],
                     w.tan[0], n, H, W, 2, seed, iter);
  DG_LAUNCH_CHECK("cnn_in_kernel<dual>");
  const unsigned int tiles = dual_grid(n, H, W);
  int cur = 0;
  for (int l = 0; l < kMid; ++l) {
    hipLaunchKernelGGL(cnn_mid_dual_kernel, dim3(tiles), dim3(kMidThreads), 0, st, w.act[l],
                       w.tan[cur], P.wm + (size_t)l * 9 * 64 * 64, P.bm + l * 64, w.act[l + 1],
                       w.tan[cur ^ 1], n, H, W);
    DG_LAUNCH_CHECK("cnn_mid_dual_kernel");
    cur ^= 1;
  }
  hipLaunchKernelGGL(cnn_out_kernel, dim3(out_grid(n, H, W)), dim3(256), 0, st, w.act[8],
                     w.tan[cur], packed, r, (const float*)nullptr, xden, xpert, n, H, W, 3, eps,
                     eps_stride, seed, iter, (double*)nullptr, 0.0);
  DG_LAUNCH_CHECK("cnn_out_kernel<dual>");
  return DG_OK;
}

dg_status cnn_launch_denoise(const dg_plan* p, const void* params, const float* r,
                             const double* eps, uint64_t seed, int iter, float* x_den,
                             float* x_pert, double* div_dot_out, hipStream_t st) {
  (void)div_dot_out;
  const dg_cnn_params* cp = (const dg_cnn_params*)params;
  CnnWork w;
  cnn_work_layout((int64_t)p->N, cp->work, &w);
  if (!x_pert) return cnn_forward(cp->weights, r, x_den, 1, p->I, p->I, w, st);
  return cnn_denoise_dual(cp->weights, r, x_den, x_pert, eps, 0, seed, iter, 1, p->I, p->I, w, st);
}

// n slices of one image size, stored back to back (r, x_den, x_pert); the
// work buffer of `params` must hold dg_cnn_workspace_bytes(n * I * I).
dg_status cnn_launch_denoise_batch(const void* params, const float* r, const double* scal_eps,
                                   int eps_stride, uint64_t seed, int iter, float* x_den,
                                   float* x_pert, int n, int I, hipStream_t st) {
  const dg_cnn_params* cp = (const dg_cnn_params*)params;
  CnnWork w;
  cnn_work_layout((int64_t)n * I * I, cp->work, &w);
  return cnn_denoise_dual(cp->weights, r, x_den, x_pert, scal_eps, eps_stride, seed, iter, n, I, I,
                          w, st);
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_cnn_weight_bytes(void) { return kPackedBytes; }
extern "C" int64_t dg_cnn_param_count(void) { return kNParams; }
extern "C" size_t dg_cnn_workspace_bytes(int64_t n_pixels) { return cnn_work_bytes(n_pixels); }

extern "C" dg_status dg_cnn_pack(const float* master, void* packed, void* stream) {
  DG_ARG_CHECK(master && packed, "dg_cnn_pack: null argument");
  hipLaunchKernelGGL(cnn_pack_kernel, dim3(g256(8 * 9 * 64 * 64)), dim3(256), 0,
                     (hipStream_t)stream, master, (char*)packed);
  DG_LAUNCH_CHECK("cnn_pack_kernel");
  return DG_OK;
}

extern "C" dg_status dg_cnn_forward(const void* packed, int32_t n, int32_t h, int32_t w,
                                    const float* in, float* out, void* work, void* stream) {
  DG_ARG_CHECK(packed && in && out && work, "dg_cnn_forward: null argument");
  DG_ARG_CHECK(n >= 1 && h >= 1 && w >= 1, "dg_cnn_forward: bad shape");
  CnnWork cw;
  cnn_work_layout((int64_t)n * h * w, work, &cw);
  return cnn_forward(packed, in, out, n, h, w, cw, (hipStream_t)stream);
}

extern "C" dg_status dg_cnn_train_step(const float* noisy, const float* clean, int32_t n,
                                       int32_t h, int32_t w, float* master, void* packed,
                                       float* grad, float* adam_m, float* adam_v, int32_t step,
                                       double lr, double* loss_out, void* work, void* stream) {
  DG_ARG_CHECK(noisy && clean && master && packed && grad && adam_m && adam_v && loss_out && work,
               "dg_cnn_train_step: null argument");
  DG_ARG_CHECK(n >= 1 && h >= 1 && w >= 1 && step >= 1 && lr > 0,
               "dg_cnn_train_step: bad shape, step or learning rate");
  hipStream_t st = (hipStream_t)stream;
  const Packed P = unpack(packed);
  CnnWork cw;
  const int64_t npix = (int64_t)n * h * w;
  cnn_work_layout(npix, work, &cw);
  dg_status rc = cnn_forward(packed, noisy, nullptr, n, h, w, cw, st);
  if (rc != DG_OK) return rc;
  // loss and dL/df
  const unsigned int gb = g256(npix);
  const unsigned int ot = out_grid(n, h, w);
  hipLaunchKernelGGL(cnn_out_kernel, dim3(ot), dim3(256), 0, st, cw.act[8], (const bf16*)nullptr,
                     packed, noisy, clean, cw.f, (float*)nullptr, n, h, w, 2, (const double*)nullptr,
                     0, (uint64_t)0, 0, cw.dpart, 1.0 / (double)npix);
  DG_LAUNCH_CHECK("cnn_out_kernel<train>");
  hipLaunchKernelGGL(cnn_loss_finish, dim3(1), dim3(256), 0, st, cw.dpart, (int)ot,
                     1.0 / (double)npix, loss_out);
  DG_LAUNCH_CHECK("cnn_loss_finish");
  // output layer: weight grads, then g8
  hipLaunchKernelGGL(cnn_small_wgrad_kernel, dim3(kWgradBlocks), dim3(256), 0, st,
                     (const bf16*)nullptr, (const float*)nullptr, cw.f, cw.act[8], cw.part, n, h, w,
                     9);
  DG_LAUNCH_CHECK("cnn_small_wgrad_kernel<9>");
  hipLaunchKernelGGL(cnn_reduce_kernel, dim3(g256(640)), dim3(256), 0, st, cw.part, kWgradBlocks,
                     640, cw.red);
  hipLaunchKernelGGL(cnn_scatter_small, dim3(g256(640)), dim3(256), 0, st, cw.red, grad, 9);
  hipLaunchKernelGGL(cnn_out_bwd_kernel, dim3(gb), dim3(256), 0, st, cw.f, packed, cw.act[8],
                     cw.tan[0], n, h, w);
  DG_LAUNCH_CHECK("cnn_out_bwd_kernel");
  const unsigned int tiles = mid_grid(n, h, w);
  int cur = 0;  // cw.tan[cur] = gradient w.r.t. the (post-ReLU-masked) output of layer l+1
  for (int l = kMid - 1; l >= 0; --l) {
    // weight gradient of mid layer l: g = tan[cur] (masked), input act[l]
    hipLaunchKernelGGL(cnn_wgrad_kernel, dim3(kWgradBlocks), dim3(256), 0, st, cw.tan[cur],
                       cw.act[l], cw.part, n, h, w);
    DG_LAUNCH_CHECK("cnn_wgrad_kernel");
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3(g256(9 * 64 * 64 + 64)), dim3(256), 0, st, cw.part,
                       kWgradBlocks, 9 * 64 * 64 + 64, cw.red);
    hipLaunchKernelGGL(cnn_scatter_mid, dim3(g256(9 * 64 * 64 + 64)), dim3(256), 0, st, cw.red,
                       grad, l);
    // data gradient into layer l's input (masked by its ReLU pattern)
    hipLaunchKernelGGL(cnn_mid_kernel<1>, dim3(tiles), dim3(kMidThreads), 0, st, cw.tan[cur],
                       P.wmt + (size_t)l * 9 * 64 * 64, (const float*)nullptr, cw.act[l],
                       cw.tan[cur ^ 1], n, h, w);
    DG_LAUNCH_CHECK("cnn_mid_kernel<bwd>");
    cur ^= 1;
  }
  // input layer
  hipLaunchKernelGGL(cnn_small_wgrad_kernel, dim3(kWgradBlocks), dim3(256), 0, st, cw.tan[cur],
                     noisy, (const float*)nullptr, (const bf16*)nullptr, cw.part, n, h, w, 0);
  DG_LAUNCH_CHECK("cnn_small_wgrad_kernel<0>");
  hipLaunchKernelGGL(cnn_reduce_kernel, dim3(g256(640)), dim3(256), 0, st, cw.part, kWgradBlocks,
                     640, cw.red);
  hipLaunchKernelGGL(cnn_scatter_small, dim3(g256(640)), dim3(256), 0, st, cw.red, grad, 0);
  // Adam and repack
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(cnn_adam_kernel, dim3(g256(kNParams)), dim3(256), 0, st, master, grad, adam_m,
                     adam_v, kNParams, (float)lr, b1, b2, 1e-8f, c1, c2);
  DG_LAUNCH_CHECK("cnn_adam_kernel");
  hipLaunchKernelGGL(cnn_pack_kernel, dim3(g256(8 * 9 * 64 * 64)), dim3(256), 0, st, master,
                     (char*)packed);
  DG_LAUNCH_CHECK("cnn_pack_kernel");
  return DG_OK;
}
