"""FP64 CPU oracle for the reduced-basis hierarchical matched filter.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(HIP kernels behind the C ABI) never calls it, and it shares no code with the
library: plain numpy/scipy (and torch CPU float64 for autograd) only.

Modules
-------
mf      the template method: strain FFT, sigma, complex SNR series, triggers,
        peaks (Sec. II, Eqs. MF_def, SNR_def, hf_eqn, IFFT).
basis   PCA/SVD basis of the whitened unit-norm bank, rank rule, coefficients,
        reduced-basis SNR (Sec. II.A, Eqs. Eq-PCA/Eq-SVD, basis_SNR,
        Beta_eqn, SNR_loss; Sec. III.B).
hier    the binned (hierarchical) first stage: bin means of the basis
        outputs, triggering bins, fine reconstruction of their samples, the
        second-stage variants, the template-method fold of Eq. avg_fft2 and
        the target SNR of Eq. target_snr_criteria (Sec. III.C-D, III.F).
stream  overlap-save segmentation of a long strain (Sec. III.E): segment
        starts, valid windows, stitched trigger lists.
nonuniform
        PCA of the bank sampled at the non-uniform frequency set (zero
        crossings of a reference template, a few frequencies per bin, a
        floor on the spacing) and linear interpolation of the basis onto the
        uniform grid (Sec. III.A, the interpolation step of Sec. III.C).
grad    loss sum g |rho|^2 over a frozen trigger set and its gradients with
        respect to the coefficients and the strain (torch CPU float64
        autograd through an independent plain forward).
"""
