"""The bound behind the scale of the FP16 FFT intermediate option: a pass-1
output of the four-step inverse transform of X = d conj(v),
Y[n2][f1] = w(f1, n2) sum_{f2 < N2} X[f1 + N1 f2] e^{2 pi i f2 n2 / N2} with a
unit twiddle w, has |Y| <= sqrt(N2) max|d| ||v|| (Cauchy-Schwarz over the
column's N2 terms), so a scale s with 2 sqrt(N2) max|d| s <= 2^15 keeps every
output of a unit-norm v below 2^14.  Random one-sided data, an adversarial v
concentrated on one column with d's phases (equality), and the scale rule's
largest output checked against the FP16 range."""
import numpy as np


def pass1_outputs(X, N1, N2):
    # column f1 holds X[f1 + N1 f2], f2 = 0..N2-1: the unnormalised inverse DFT down each column
    return np.fft.ifft(X.reshape(N2, N1), axis=0) * N2


def scale_rule(dmax, N2):
    bound = 2.0 * np.sqrt(N2) * dmax
    e = 0 if bound == 0 else int(np.floor(np.log2(32768.0 / bound)))
    return 2.0 ** max(-120, min(120, e))


def test_bound_random_and_adversarial():
    rng = np.random.default_rng(2110)
    for N1, N2 in ((64, 64), (256, 128), (2048, 256)):
        N = N1 * N2
        for _ in range(3):
            d = (rng.normal(size=N) + 1j * rng.normal(size=N)) * rng.uniform(0.1, 1e3)
            d[N // 2:] = 0.0                       # one-sided band, as the correlation prologue reads it
            v = rng.normal(size=N) + 1j * rng.normal(size=N)
            v[N // 2:] = 0.0
            v /= np.linalg.norm(v)
            Y = pass1_outputs(d * np.conj(v), N1, N2)
            bound = np.sqrt(N2) * np.abs(d).max()
            assert np.abs(Y).max() <= bound * (1 + 1e-12)
            s = scale_rule(np.abs(d).max(), N2)
            assert np.abs(Y).max() * s <= 2.0 ** 14 and np.abs(Y).max() * s < 65504.0
        # equality: v on one column with unit-modulus d aligned in phase, |d| = D everywhere
        D, f1 = 7.5, 3
        ph = rng.uniform(0, 2 * np.pi, size=N)
        d = D * np.exp(1j * ph)
        v = np.zeros(N, complex)
        idx = f1 + N1 * np.arange(N2)
        v[idx] = np.exp(1j * ph[idx]) / np.sqrt(N2)
        Y = pass1_outputs(d * np.conj(v), N1, N2)
        assert np.isclose(np.abs(Y).max(), np.sqrt(N2) * D, rtol=1e-12)
        assert np.abs(Y).max() * scale_rule(D, N2) <= 2.0 ** 14


def test_scale_rule_edges():
    assert scale_rule(0.0, 256) == 1.0            # all-zero data: no scaling
    assert scale_rule(1e-40, 256) == 2.0 ** 120   # extreme data: the exponent is clamped
    assert scale_rule(1e40, 256) == 2.0 ** -120
    s = scale_rule(3.0, 256)                       # the largest power of two under the rule
    assert 2 * 16 * 3.0 * s <= 32768.0 < 2 * 16 * 3.0 * 2 * s
