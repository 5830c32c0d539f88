"""FP64 CPU oracle for joint time-frequency scattering (JTFS) and its gradient.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
anything under this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP path
(no kernels, headers, tables or constants generators): the only module both sides
read is ``jtfs_inputs``, which draws seeded signals and holds no transform arithmetic.

Contents
--------
filterbank  Morlet / Gaussian filters (paper Eq. 1, Sec. 3.1 generator, Sec. 3.4 spin)
            in the Fourier domain (periodised closed form) and in the time domain
            (periodised continuous Morlet), plus the subsampling-scale rule.
plan        Filterbanks, subsampling factors, second-order pairs, frequential filter
            list and output layout (Sec. 3.1-3.5), derived independently of the C++ plan.
fftroute    "O2": forward transform through FFTs, Fourier-domain filtering and
            Fourier subsampling, as the paper's implementation does (Sec. 3.2-3.5,
            Eqs. 2-4), and the exact hand-written adjoint (Sec. 2.3, Eqs. 5-7).
brute       "O1": the same transform by direct circular convolutions with
            time-domain filters and index-stride decimation (tiny sizes only).
descent     Loss, relative loss and the metamer updates (Sec. 2.3): gradient
            descent, Adam, and momentum with the bold-driver learning rate.
init        The paper's descent start (Sec. 2.3): Gaussian noise whose power spectral
            density matches S1 x (band levels, Rayleigh factor, the interpolated
            spectrum and the shaping of given standard normal draws).
figure      The joint time--log-frequency wavelet of a path (Sec. 2.1, Fig. 1): the real
            part of psi_alpha(t) psi_beta(log2 lambda) from the time-domain filters.
decoder     The learned warm start (an addition to the method, not in the paper): a
            1-D transposed-convolution decoder from coefficients to a waveform, its
            exact adjoint with the device's bfloat16 storage points, and Adam.

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``
except the conventions listed as "parity unpinned" in ``plan`` (the widths of
phi_T / phi_F, the subsampling-scale constant, padding and frequential padding
length, which coefficients enter the loss); those are readings of the paper, not
results it fixes.
"""
