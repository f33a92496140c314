"""The persistent FMA stage kernel (single propagations with N <= 16 and at
least 32768 ADOs) against the FP64 oracle.

Every ADO starts from random values, so that every coupling line (the "-"
rows of all levels, sigma_0 as the "-" neighbour of level 1, the "+" rows
below the top level) carries weight from the first step; three RK4 steps are
compared element by element over the whole hierarchy.  Tolerances: FP64 1e-12
of the largest element; FP32-mixed 2e-5 of it (each stage rounds every
stored element once, 12 stages give ~1e-6, and sums over up to W + D
neighbours of comparable scale cancel).
"""

import numpy as np
import pytest

import heom_inputs as hi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def heom():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_03498_amd as heom
    heom.load()
    return heom


def _case(*args):
    print("CASE", *args, flush=True)


CASES = [
    # name, seed, N, M, D, Hermitian, complex H
    ("N8_W16_D6_herm", 71, 8, 1, 6, True, False),
    ("N7_W14_D6_nonherm", 72, 7, 1, 6, False, False),
    ("N5_W15_D6_complexH", 73, 5, 2, 6, True, True),
]


@pytest.mark.parametrize("name,seed,N,M,D,herm,cplx", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_small_kernel_matches_oracle(heom, orc, name, seed, N, M, D, herm, cplx, precision):
    _case("small kernel", name, precision)
    prob = hi.random_problem(seed, N, M=M, D=D, complex_h=cplx)
    W, n = orc.sizes(prob)
    assert n >= 32768
    x0 = hi.random_state(seed + 100, n, N, hermitian=herm, scale=0.1)
    x0[0] = hi.population_rho0(N, N // 2) if herm else x0[0]
    y_ref, rec_ref = orc.propagate(prob, x0, 0.5, 3, 1)
    h = heom.Hierarchy(prob, precision)
    st = h.state_from_numpy(x0)
    rec = h.propagate(st, 0.5, 3, 1, hermitian=herm)
    y = h.state_to_numpy(st)
    scale = np.max(np.abs(y_ref))
    tol = 1e-12 if precision == 0 else 2e-5
    err = np.max(np.abs(y - y_ref))
    print("  max error / max element %.3e" % (err / scale), flush=True)
    assert err <= tol * scale
    assert np.max(np.abs(rec[:, :N] - rec_ref[:, :N])) <= tol * max(1.0, np.max(np.abs(rec_ref[:, :N])))


def test_small_kernel_n16_fp64_matches_oracle(heom, orc):
    # N = 16: N^2 = 256, the largest divisor of the kernel's index decode;
    # eight baths at depth 10 (43758 ADOs), FP64 (FP32 at N >= 10 takes the
    # matrix-core kernel); one RK4 step (all four stage forms) against the
    # oracle element by element
    _case("small kernel N16 fp64")
    prob = hi.random_problem(74, 16, n_baths=8, M=0, D=10)
    W, n = orc.sizes(prob)
    assert W == 8 and n == 43758
    x0 = hi.random_state(174, n, 16, hermitian=True, scale=0.1)
    x0[0] = hi.population_rho0(16, 8)
    y_ref, rec_ref = orc.propagate(prob, x0, 0.5, 1, 1)
    h = heom.Hierarchy(prob, 0)
    st = h.state_from_numpy(x0)
    rec = h.propagate(st, 0.5, 1, 1, hermitian=True)
    y = h.state_to_numpy(st)
    scale = np.max(np.abs(y_ref))
    err = np.max(np.abs(y - y_ref))
    print("  max error / max element %.3e" % (err / scale), flush=True)
    assert err <= 1e-12 * scale
    assert np.max(np.abs(rec[:, :16] - rec_ref[:, :16])) <= 1e-12 * max(1.0, np.max(np.abs(rec_ref[:, :16])))
