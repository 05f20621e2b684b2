"""FP64 CPU oracle for the D-GAMP-CT hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import anything in this
package.  It shares no code, headers, tables or helpers with the GPU library
(``paper_1609_04661_amd``), and it never imports it.

Every function follows a passage of Perelli, Lexa, Can & Davies,
"Compressive CT reconstruction through Denoising Approximate Message
Passing" (arXiv 1609.04661), cited by section / equation / algorithm:

  geometry   ray lines of the parallel and fan acquisitions (Sec. 2.1)
  radon      exact-chord system matrix A and A^T (Sec. 2.1, eq. linCT)
  precond    cone preconditioner V, V^-1 (Sec. 2.4, eqs. PPFT preconditioner,
             Aprecon, GramATA)
  channel    Poisson output channel of GAMP: mode, Laplace moments, s, tau_s
             (Sec. 4.2, eqs. MMSEmm / post_exp, Appendix A)
  denoisers  Haar soft threshold and non-local means plug-ins, and the
             Monte-Carlo divergence (Sec. 4.3, eq. MC_SURE)
  probe      the counter-based Rademacher probe (SplitMix64)
  gamp       the GAMP recursion of Algorithm 1 and its pins (AWGN channel,
             Bernoulli-Gaussian MMSE denoiser, state evolution, Sec. 3/4.4)
  cnn        FP64 forward / backward / tangent of the residual CNN denoiser
  metrics    PSNR / SSIM (Sec. 6)

Each module's docstring states the parity status (pinned / unpinned) of its
functions and what pins them.
"""
