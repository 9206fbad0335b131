"""FP64 CPU oracle for overlapping-domain-decomposition ptychography (OD2P / OD2Pm / OD2BP).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy (complex128) statement of what the GPU library computes, written from the
paper's equations.  Only the test-suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product library never calls it and it never
calls the product library.  It shares no code with the GPU path: its index maps,
operators, proximal map and iterations are written here independently.

Modules
-------
geometry   subdomains, restrictions, pair sets, overlap multiplicities (Sec. 2.1, 3.1)
operators  unitary 2-D DFT, window S_j, forward A and adjoint A*, diag(A*A) (Sec. 2, eq. AtA)
stagm      ST-AGM metric, gradient and closed-form proximal map (Sec. 2.2)
od2p       Algorithm 2 (OD2Pm; Algorithm 1 is D=2), an undecomposed ADMM, merge, RF/RE/SNR,
           augmented Lagrangian (Sec. 2.3, 3.1, 4)
blind      Algorithm 3 (OD2BP) with the probe-support projection (Sec. 3.2)
amploss    amplitude data-term loss and its gradient in u and w
local      one iteration of Algorithm 2 or 3 on chosen subdomains only (sampled checks at
           full problem sizes)
balance    overlap penalty r chosen by residual balancing (future work of Sec. 4.3 and 5;
           He, Yang and Wang 2000; Boyd et al. 2011, Sec. 3.4.1)
"""
