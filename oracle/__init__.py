"""FP64 CPU oracle for the PSWF-LR reciprocal-space path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only the test suite, the smoke
check and the CPU-baseline leg of the benchmark do.  The oracle shares no code
with the HIP path (no kernels, headers, helpers, tables or constants): it is a
plain, slow, obviously correct re-statement of the paper's definitions.

Modules
-------
pswf        order-zero prolate spheroidal wave function psi_0^c (Methods,
            "Prolate spheroidal wave functions"), by the Legendre-tridiagonal
            method for the prolate differential operator.
kernels     mollifiers G_p (Eqs. G1, G6, G), Fourier kernels Phi_p (Eq. PhiH),
            self terms and zero-frequency terms (Methods, "Implementation
            details").
reciprocal  direct structure-factor sum of the truncated Fourier energy
            (Eq. Fourier) with potentials, forces and virial.
cellsum     the same Fourier sum for a general (triclinic) cell H, structure
            factors from separable phase tables in fractional coordinates,
            potentials and forces for a sample of atoms (large structures).
realspace   real-space complement (1 - G_p)/r^p summed over images.
ewald       textbook Ewald for p = 1 (independent cross-check only; Eq.
            screening).
brute       brute-force periodic image sums for p > 3.
mesh        the paper's four-step mesh algorithm (Methods, "Accelerating
            atom-grid spreading with PSWFs") in plain form, for stage-level
            parity: spread, FFT, diagonal scaling, reduction, and the adjoint
            gather.

Parity status of every function is listed in its module header; anything
not pinned against something other than itself says "parity unpinned".
"""
