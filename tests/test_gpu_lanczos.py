"""Block Lanczos basis (rb_build_basis_solver, RB_EIG_LANCZOS) against the
oracle: eigenvalues of the T x T Gram matrix of the whitened unit templates
(numpy.linalg.eigh, FP64) and the leading right singular subspace
(numpy.linalg.svd), both of the templates as the library stores them
(complex64, rounded once from FP64: the operand its products read), and
against the subspace-iteration basis.  The search with the Lanczos basis
must give the oracle's trigger set."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from paper_2110_13115_amd import rbmf
from tests.helpers import Case, compare_triggers

pytestmark = pytest.mark.gpu


def log(*a):
    print("[gpu-lanczos]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lz():
    case = Case(N=32768, T=420, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=61,
                inj=((11, 12.0), (200, 8.0)))
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    W, _ = case.whitened()
    W32 = W.astype(np.complex64).astype(np.complex128)
    lam_ref = np.sort(np.linalg.eigvalsh(W32 @ W32.conj().T))[::-1]
    _, so, Vh = np.linalg.svd(W32, full_matrices=False)
    yield case, ctx, bank, W32, lam_ref, Vh
    bank.close()


def orthonormal_rows(V):
    """Rows spanning the same space as V's, orthonormal in FP64 (QR)."""
    Q, _ = np.linalg.qr(V.conj().T)
    return Q.conj().T


def subspace_sin(A, B):
    """Largest principal-angle sine between the row spaces of A and B (orthonormal rows)."""
    sv = np.linalg.svd(A @ B.conj().T, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - sv.min() ** 2)))


@pytest.mark.parametrize("rank", [0, 60])
def test_lanczos_basis_vs_oracle(lz, rank):
    case, ctx, bank, W32, lam_ref, Vh = lz
    lb = rbmf.Basis(ctx, bank, rank=rank, tol=1e-3, dtype="f32", solver="lanczos")
    sb = rbmf.Basis(ctx, bank, rank=rank, tol=1e-3, dtype="f32", solver="subspace")
    try:
        check_lanczos(case, ctx, bank, W32, lam_ref, Vh, rank, lb, sb)
    finally:
        lb.close()
        sb.close()


def check_lanczos(case, ctx, bank, W32, lam_ref, Vh, rank, lb, sb):
    K = lb.K
    cum = np.cumsum(lam_ref) / np.sum(lam_ref)
    K_ref = rank if rank else int(np.searchsorted(cum, 1 - 1e-3 - 1e-15) + 1)
    assert K == K_ref == sb.K
    V, c, lam = lb.export()
    Vs, cs, lams = sb.export()
    rel = np.abs(lam - lam_ref[:K]) / lam_ref[:K]
    log(f"rank {rank}: K {K}, eigenvalue rel err max {rel.max():.2e} (subspace iteration "
        f"{(np.abs(lams - lam_ref[:K]) / lam_ref[:K]).max():.2e}), lambda_K / lambda_1 {lam_ref[K - 1] / lam_ref[0]:.2e}")
    assert rel.max() <= 1e-8
    # stored basis rows are complex64, orthonormal only to ~1e-8: re-orthonormalise them in FP64
    # before measuring the angle (sqrt(1 - cos^2) of a cosine that is 1 - 1e-8 from rounding alone
    # would read as a sine of 1.4e-4)
    gap = (lam_ref[K - 1] - lam_ref[K]) / lam_ref[0]
    sin_l = subspace_sin(Vh[:K], orthonormal_rows(V))
    sin_s = subspace_sin(Vh[:K], orthonormal_rows(Vs))
    log(f"  subspace sine vs oracle {sin_l:.2e} (subspace iteration {sin_s:.2e}; relative gap at K {gap:.2e})")
    assert sin_l <= 1e-6 + 1e-9 / gap
    assert sin_s <= 1e-6 + 1e-9 / gap
    np.testing.assert_allclose(c, W32 @ V.conj().T, atol=2e-6)
    assert abs(lb.energy - sb.energy) <= 1e-9
    # same search result as the oracle
    trig, _, _ = rbmf.rb_filter(ctx, lb, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_SPARSE)
    compare_triggers(trig, case.rho, 6.0)


def test_lanczos_sub_bank_and_full_rank(lz):
    """A sub-bank range, and a rank equal to the sub-bank's size (the Krylov
    space reaches T: exact reconstruction)."""
    case, ctx, bank, W32, lam_ref, Vh = lz
    t0, t1 = 100, 160
    lb = rbmf.Basis(ctx, bank, rank=t1 - t0, dtype="f32", t0=t0, t1=t1, solver="lanczos")
    V, c, lam = lb.export()
    Ws = W32[t0:t1]
    ref = np.sort(np.linalg.eigvalsh(Ws @ Ws.conj().T))[::-1]
    np.testing.assert_allclose(lam, ref, rtol=1e-7, atol=1e-12 * ref[0])
    assert np.abs(c @ V - Ws).max() <= 1e-5
    lb.close()
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.lib()
        import ctypes as C
        h = C.c_void_p()
        rbmf._check(rbmf.lib().rb_build_basis_solver(ctx.h, bank.h, 0, 10, 3, 1e-3, 0, 7, C.byref(h), None, None),
                    "rb_build_basis_solver")
    assert ei.value.status == rbmf.RB_ERR_ARG
