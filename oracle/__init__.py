"""CPU FP64 oracle for the MLFMA-SMR hot path -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference the HIP library
is checked against.  It computes the *definition* of what the fast
matrix-vector product approximates: the dense static-mode PMCHWT operator
(Sec. II, eqs. PMCHWT, Zpq_delta, PMCHWT_Finite1, BasisTransformation) with
its entries from direct quadrature, the static modes it is expressed in
(Sec. III, eqs. AuxProb_Tl/Operator_Tlo and AuxProb_Tt/Operator_Tto), the
plane-wave right-hand side, a dense solve, and the scattered fields.  It does
not run the multilevel fast multipole algorithm.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The library under
``paper_2407_21724_amd`` shares no code with it; the only common inputs come
from the seeded generators in ``workloads``.

Conventions (readings of the paper, each listed in the design notes):
  * time dependence exp(+j w t); g = exp(-j k R) / (4 pi R)   (Sec. II)
  * lengths in background wavelengths, k- = 2 pi, eps- = mu = 1, zeta- = 1
  * electric current j_e = n x H, magnetic current j_m = E x n
  * T_mn = <psi_m, L psi_n> with L the field operator of an electric
    current divided by zeta:  L u = -jk int g u + (1/(jk)) grad int g div'u
    (the dyadic form of eq. T_far1);
    K_mn = <psi_m, int psi_n x grad g>  (gradient on the observation point;
    this is the sign under which eq. Kmn_fmm follows from eq. addition_th)
  * Z^{mu nu} as in eq. Zpq_delta with these T and K, and
    V = -[<psi, E_inc>; <psi, H_inc>].

Functions without an independent pin say "parity unpinned" in their
docstring.
"""
