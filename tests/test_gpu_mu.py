"""The multiplicative-update baseline (nmf_mu_sweep) against the FP64 MU
oracle (MI355X only): the same bars as the FAST-HALS path -- relative
objective within 1e-5 of the oracle's after every sweep, factors within 1e-3
(relative Frobenius) after 10 sweeps -- plus the paper's qualitative claim
(Sec. 6.3) that FAST-HALS reaches a lower objective than MU in as many sweeps."""
import numpy as np
import pytest

import datagen
from oracle import hals, mu
from tests.gpu_util import EPS, col_rel_max, gpu_plan, oracle_A, rel_fro, small_bow, sparse_init

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def _oracle_mu(A, W0, H0, sweeps):
    Ao = oracle_A(A)
    W, H = hals.normalize_columns(W0), H0.astype(np.float64)
    rels, facs = [], []
    for _ in range(sweeps):
        W, H = mu.mu_sweep(Ao, W, H, EPS)
        rels.append(hals.objective(Ao, W, H)[1])
        facs.append((W.copy(), H.copy()))
    return np.array(rels), facs


@pytest.mark.parametrize("case", ["dense", "sparse", "dense_k33"])
def test_mu_matches_oracle(cuda, case):
    if case == "sparse":
        c = small_bow()
        A, K = c.A, 24
        W0, H0 = sparse_init(c, K)
    else:
        K = 33 if case == "dense_k33" else 16
        A = datagen.dense_planted_uniform(400, 300, 12, 0.01, seed=3)
        W0, H0 = datagen.uniform_init(400, 300, K, seed=1)
    plan = gpu_plan(A, W0, H0, cuda)
    rel = []
    for i in range(20):
        rel += plan.mu_sweep(1, objective=True)
        if i == 9:
            W10, H10 = _np(plan.W), _np(plan.Ht).T
    plan.close()
    ref, facs = _oracle_mu(A, W0, H0, 20)
    d = np.abs(np.array(rel) - ref) / ref
    assert d.max() <= 1e-5, d
    assert rel_fro(W10, facs[9][0]) <= 1e-3 and rel_fro(H10, facs[9][1]) <= 1e-3
    assert col_rel_max(W10, facs[9][0]) <= 2e-3
    # MU never increases the objective (up to FP32 rounding)
    assert np.all(np.diff(rel) <= 1e-6 * np.array(rel[1:]))


def test_hals_beats_mu_in_equal_sweeps(cuda):
    c = small_bow()
    K = 24
    W0, H0 = sparse_init(c, K)
    ph = gpu_plan(c.A, W0, H0, cuda)
    pm = gpu_plan(c.A, W0, H0, cuda)
    rh = ph.sweep(20, objective=True)
    rm = pm.mu_sweep(20, objective=True)
    ph.close()
    pm.close()
    assert rh[-1] < rm[-1]
    assert all(h <= m for h, m in zip(rh[4:], rm[4:]))
