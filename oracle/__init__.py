"""FP64 CPU oracle for the sparse w-projection measurement operator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU path computes.  It exists to judge
the HIP library: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it.  It shares no code, tables or constants
with the HIP path and never imports it.

Paper: Wolz, McEwen, Abdalla, Carrillo & Wiaux (2013), "Revisiting the spread
spectrum effect in radio interferometric imaging: a sparse variant of the
w-projection algorithm".  Each function cites the passage it follows.

Modules
-------
geometry    pixel / grid coordinates of the padded grid (Sections 2.2, 4.1)
kb          Kaiser-Bessel window, its Fourier transform and the gridding taps
chirp       exact w-modulation (Eq. 4) and its linear chirp (Eq. 5)
wproj       kernel rows (chirp FT convolved with KB, Section 3.1), energy
            sparsification (Section 3.2), CSR assembly and Phi / Phi-adjoint
dft         brute-force direct evaluation of the measurement equation (Eq. 1/3)
paper_form  the paper's own on-grid operator C-hat F U (Eq. 8) for the
            non-zero-fraction check of Section 3.2
wavelet     Daubechies-8 filters by spectral factorisation and a periodic DWT
solver      primal-dual solver of the constrained l1 problem (Eq. 7)
metrics     SNR definitions of Section 4.1

Parity status per function is listed in each module header; a function whose
result no pin fixes says "parity unpinned".
"""
