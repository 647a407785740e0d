"""Fold-in (H-only FAST-HALS with W fixed) and the warm-start network on the
GPU, against the FP64 oracle (MI355X only).

The network's products take BF16 operands with FP32 accumulation; the oracle
is evaluated at the same BF16-rounded weights and inputs, and the remaining
difference (BF16 rounding of the hidden activations and of the backward
intermediates) is held to the stated tolerances."""
import numpy as np
import pytest

import datagen
from oracle import hals
from oracle import mlp as omlp
from tests.gpu_util import (EPS, bf16_round, gpu_plan, oracle_A, rel_fro, rows_csr_to_oracle,
                            small_bow, sparse_init)

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def _fold_setup(cuda, K=16, sweeps=5, Dn=400, seed=7):
    """Oracle W after a few sweeps, a plan carrying that W, and new documents."""
    c = small_bow(2000, 900)
    W0, H0 = sparse_init(c, K)
    Ao = oracle_A(c.A)
    W = hals.normalize_columns(W0)
    H = H0.astype(np.float64)
    for _ in range(sweeps):
        W, H = hals.sweep(Ao, W, H, EPS)
    new = datagen.bag_of_words_docs(Dn, 1.1, 77.0, seed, c.perm, c.idf)
    plan = gpu_plan(c.A, W.astype(np.float32), H.astype(np.float32), cuda)
    return c, W, new, plan


@pytest.mark.parametrize("K", [16, 200])
def test_foldin_given_init_matches_oracle(cuda, K):
    """K = 200 is the fold-in workload's rank (the wide sparse-product kernel)."""
    import torch

    from paper_1904_07935_amd.api import Matrix
    c, W, new, plan = _fold_setup(cuda, K=K)
    K, Dn = W.shape[1], new.rows
    Anew = rows_csr_to_oracle(new)
    _, H0 = datagen.uniform_init_matched(c.A.rows, Dn, K, datagen.mean_value(new), seed=4)
    Ht = torch.tensor(np.ascontiguousarray(H0.T), device=cuda)
    trace = plan.foldin(Matrix.from_csr(new, cuda), Ht, init="given", n_sweeps=20)
    rels = [hals.objective(Anew, W, H0.astype(np.float64))[1]]
    Ho = hals.foldin(Anew, W, H0, EPS, 20,
                     on_sweep=lambda i, H: rels.append(hals.objective(Anew, W, H)[1]))
    d = np.abs(np.array(trace) - np.array(rels)) / np.array(rels)
    assert d.max() <= 1e-5, d
    assert rel_fro(_np(Ht).T, Ho) <= 1e-4
    # the objective of an H-only sweep never increases
    assert np.all(np.diff(trace) <= 1e-6 * np.array(trace[1:]))
    plan.close()


def test_foldin_tolerance_stop(cuda):
    """With tol > 0 fold-in stops after the first sweep that lowers the relative
    objective by less than tol; the sweeps it ran are the same sweeps a
    fixed-count run performs (bitwise), and the count is reported."""
    import torch

    from paper_1904_07935_amd.api import Matrix
    c, W, new, plan = _fold_setup(cuda, K=16)
    Dn, K = new.rows, W.shape[1]
    _, H0 = datagen.uniform_init_matched(c.A.rows, Dn, K, datagen.mean_value(new), seed=4)
    M = Matrix.from_csr(new, cuda)
    tol = 1e-6
    Ht = torch.tensor(np.ascontiguousarray(H0.T), device=cuda)
    tr = plan.foldin(M, Ht, init="given", n_sweeps=300, tol=tol)
    n = plan.foldin_sweeps
    assert 1 <= n < 300 and len(tr) == n + 1
    dec = -np.diff(tr)
    assert dec[-1] < tol and np.all(dec[:-1] >= tol), dec
    Ht2 = torch.tensor(np.ascontiguousarray(H0.T), device=cuda)
    tr2 = plan.foldin(M, Ht2, init="given", n_sweeps=n)
    assert plan.foldin_sweeps == n
    assert torch.equal(Ht, Ht2)
    np.testing.assert_array_equal(tr, tr2)
    plan.close()


def test_foldin_wta_init_is_clipped_projection(cuda):
    import torch

    from paper_1904_07935_amd.api import Matrix
    c, W, new, plan = _fold_setup(cuda, K=12)
    Anew = rows_csr_to_oracle(new)
    Ht = torch.zeros(new.rows, W.shape[1], device=cuda)
    plan.foldin(Matrix.from_csr(new, cuda), Ht, init="wta", n_sweeps=0, trace=False)
    ref = np.maximum(EPS, np.asarray(Anew.T @ W))
    assert rel_fro(_np(Ht), ref) <= 1e-5
    plan.close()


def _net(rng, K, H):
    return {"W1": rng.normal(size=(H, K)) / np.sqrt(K), "b1": 0.1 * rng.normal(size=H),
            "W2": rng.normal(size=(K, H)) / np.sqrt(H), "b2": 0.1 * rng.normal(size=K)}


def _bf16_params(p):
    q = dict(p)
    q["W1"] = bf16_round(p["W1"])
    q["W2"] = bf16_round(p["W2"])
    q["b1"] = np.asarray(p["b1"], dtype=np.float32).astype(np.float64)
    q["b2"] = np.asarray(p["b2"], dtype=np.float32).astype(np.float64)
    return q


def test_mlp_forward_and_warm_start_match_oracle(cuda):
    import torch

    from paper_1904_07935_amd.api import Matrix, Mlp
    rng = np.random.default_rng(0)
    K, Hd, N = 16, 64, 300
    p = _net(rng, K, Hd)
    net = Mlp(K, Hd, device=cuda, seed=None)
    net.set_masters(p)
    X = rng.random((N, K)).astype(np.float32)
    Y = _np(net.forward(torch.tensor(X, device=cuda)))
    yo, _ = omlp.forward(_bf16_params(p), bf16_round(X))
    assert rel_fro(Y, yo) <= 1e-2
    # the fold-in warm start: network on normalised rows of A_new^T W, rescaled
    c, W, new, plan = _fold_setup(cuda, K=K)
    Anew = rows_csr_to_oracle(new)
    Ht = torch.zeros(new.rows, K, device=cuda)
    plan.foldin(Matrix.from_csr(new, cuda), Ht, init="mlp", mlp=net, n_sweeps=0, trace=False)
    h0 = omlp.warm_start(_bf16_params(p), np.asarray(Anew.T @ W), EPS)
    assert rel_fro(_np(Ht), h0) <= 2e-2
    plan.close()


@pytest.mark.parametrize("K,Hd,Dn", [(200, 512, 1000), (40, 96, 300), (8, 32, 257)])
def test_fused_warm_start_matches_oracle_and_two_gemm_route(cuda, K, Hd, Dn):
    """Fold-in's warm start runs as one fused kernel (x in registers, the hidden
    layer through LDS, softplus, rescaling and the clip in the output
    epilogue).  Against the FP64 oracle at the same BF16-rounded weights, and
    element by element against the network's two-GEMM inference
    (nmf_mlp_predict) on the same rows: the configured size, other hidden
    widths (3 and 1 chunks of 32), row counts that leave the last 256-row
    workgroup partly empty, and K = 8 (one 16-wide step, half of it padding)."""
    import torch

    from paper_1904_07935_amd.api import Matrix, Mlp
    rng = np.random.default_rng(K + Hd)
    p = _net(rng, K, Hd)
    net = Mlp(K, Hd, device=cuda, seed=None)
    net.set_masters(p)
    c, W, new, plan = _fold_setup(cuda, K=K, Dn=Dn, sweeps=3)
    M = Matrix.from_csr(new, cuda)
    Ht = torch.zeros(new.rows, K, device=cuda)
    plan.foldin(M, Ht, init="mlp", mlp=net, n_sweeps=0, trace=False)
    got = _np(Ht)
    assert np.all(np.isfinite(got)) and got.min() >= EPS * (1 - 1e-6)
    Anew = rows_csr_to_oracle(new)
    h0 = omlp.warm_start(_bf16_params(p), np.asarray(Anew.T @ W), EPS)
    assert rel_fro(got, h0) <= 2e-2
    # the two-GEMM route on the library's own rows of A_new^T W
    R = torch.zeros(new.rows, K, device=cuda)
    plan.foldin(M, R, init="wta", n_sweeps=0, trace=False)  # max(eps, A_new^T W)
    nrm = R.norm(dim=1, keepdim=True)
    y = net.forward(R / nrm)
    ref = _np(torch.clamp(nrm * y, min=EPS))
    assert rel_fro(got, ref) <= 1e-3
    d = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-6 * np.abs(ref).max())
    assert d.max() <= 3e-2
    plan.close()


def test_mlp_gradients_match_oracle(cuda):
    import torch

    from paper_1904_07935_amd.api import Mlp
    rng = np.random.default_rng(1)
    K, Hd, N = 24, 64, 256
    p = _net(rng, K, Hd)
    net = Mlp(K, Hd, device=cuda, seed=None)
    net.set_masters(p)
    X = rng.random((N, K)).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Yt = rng.random((N, K)).astype(np.float32)
    loss, grads, _ = net.loss_grad(torch.tensor(X, device=cuda), torch.tensor(Yt, device=cuda))
    lo, go = omlp.loss_and_grads(_bf16_params(p), bf16_round(X), Yt.astype(np.float64))
    assert abs(loss - lo) <= 1e-2 * lo
    for k in ("W1", "b1", "W2", "b2"):
        assert rel_fro(_np(grads[k]), go[k]) <= 5e-2, k


def test_mlp_configured_size_matches_oracle(cuda):
    """The warm-start network at its configured size (K = 200 -> 512 -> 200):
    forward and gradients against the FP64 oracle at the same BF16-rounded
    weights and inputs, on a batch of 2048 normalised inputs."""
    import torch

    from paper_1904_07935_amd.api import Mlp
    rng = np.random.default_rng(4)
    K, Hd, N = 200, 512, 2048
    p = _net(rng, K, Hd)
    net = Mlp(K, Hd, device=cuda, seed=None)
    net.set_masters(p)
    X = rng.random((N, K)).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Yt = (0.05 * rng.random((N, K))).astype(np.float32)
    Y = _np(net.forward(torch.tensor(X, device=cuda)))
    yo, _ = omlp.forward(_bf16_params(p), bf16_round(X))
    assert rel_fro(Y, yo) <= 1e-2
    loss, grads, _ = net.loss_grad(torch.tensor(X, device=cuda), torch.tensor(Yt, device=cuda))
    lo, go = omlp.loss_and_grads(_bf16_params(p), bf16_round(X), Yt.astype(np.float64))
    assert abs(loss - lo) <= 1e-2 * lo
    for k in ("W1", "b1", "W2", "b2"):
        assert rel_fro(_np(grads[k]), go[k]) <= 5e-2, k


def test_adam_step_matches_oracle(cuda):
    import torch

    from paper_1904_07935_amd.api import Mlp
    rng = np.random.default_rng(2)
    K, Hd = 8, 32
    p = _net(rng, K, Hd)
    net = Mlp(K, Hd, device=cuda, seed=None)
    net.set_masters(p)
    po = {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in p.items()}
    st = {}
    for step in range(3):
        g = {k: rng.normal(size=np.shape(v)) for k, v in p.items()}
        flat = np.concatenate([np.asarray(g[k], dtype=np.float32).ravel() for k in ("W1", "b1", "W2", "b2")])
        net.adam_step(torch.tensor(flat, device=cuda), lr=1e-2)
        omlp.adam_step(po, {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in g.items()},
                       st, lr=1e-2)
        m = net.masters()
        for k in po:
            assert rel_fro(_np(m[k]), po[k]) <= 1e-6, (step, k)


def test_trained_warm_start_beats_cold_start(cuda):
    """The learned part's gain: trained on (normalised A^T W rows -> converged
    fold-in solutions) that HALS itself produced, the network's warm start needs
    fewer H-only sweeps than both the cold start and the non-learned WTA start
    (max(eps, A^T W)) to come within 1e-4 of the cold start's converged
    relative objective on held-out documents."""
    import torch

    from paper_1904_07935_amd.api import Matrix, Mlp
    c = small_bow(3000, 1200)
    K = 20
    W0, H0 = sparse_init(c, K)
    plan = gpu_plan(c.A, W0, H0, cuda)
    plan.sweep(30)
    train = datagen.bag_of_words_docs(6000, 1.1, 77.0, 3, c.perm, c.idf)
    evald = datagen.bag_of_words_docs(1000, 1.1, 77.0, 5, c.perm, c.idf)
    Mtr, Mev = Matrix.from_csr(train, cuda), Matrix.from_csr(evald, cuda)

    def cold(n):
        _, h = datagen.uniform_init_matched(c.A.rows, n.rows, K, datagen.mean_value(n), seed=4)
        return torch.tensor(np.ascontiguousarray(h.T), device=cuda)

    # training pairs from HALS itself
    Hstar = cold(train)
    plan.foldin(Mtr, Hstar, init="given", n_sweeps=200, trace=False)
    R = torch.zeros(train.rows, K, device=cuda)
    plan.foldin(Mtr, R, init="wta", n_sweeps=0, trace=False)
    nrm = R.norm(dim=1, keepdim=True)
    X, Y = R / nrm, Hstar / nrm
    net = Mlp(K, 128, device=cuda, seed=11)
    losses = net.train(X, Y, epochs=40, batch=256, lr=2e-3, seed=3)
    assert losses[-1] < 0.5 * losses[0]

    # held-out documents: sweeps to come within 1e-4 of the converged objective
    ref = plan.foldin(Mev, cold(evald), init="given", n_sweeps=400)
    target = ref[-1] + 1e-4
    tr_cold = plan.foldin(Mev, cold(evald), init="given", n_sweeps=100)
    tr_mlp = plan.foldin(Mev, torch.zeros(evald.rows, K, device=cuda), init="mlp", mlp=net,
                         n_sweeps=100)
    tr_wta = plan.foldin(Mev, torch.zeros(evald.rows, K, device=cuda), init="wta", n_sweeps=100)

    def sweeps_to(tr, gap=1e-4):
        hit = [i for i, v in enumerate(tr) if v <= ref[-1] + gap]
        return hit[0] if hit else 10 ** 9

    s_cold, s_mlp, s_wta = sweeps_to(tr_cold), sweeps_to(tr_mlp), sweeps_to(tr_wta)
    print(f"sweeps to target: cold {s_cold}, wta {s_wta}, mlp {s_mlp}; rel0 cold {tr_cold[0]:.5f} "
          f"wta {tr_wta[0]:.5f} mlp {tr_mlp[0]:.5f}")
    for gap in (1e-5, 1e-6, 1e-7):
        print(f"  within {gap:g}: cold {sweeps_to(tr_cold, gap)} wta {sweeps_to(tr_wta, gap)} "
              f"mlp {sweeps_to(tr_mlp, gap)}")
    assert tr_mlp[0] < tr_cold[0] and tr_mlp[0] < tr_wta[0]
    assert s_mlp < s_cold and s_mlp < s_wta
    plan.close()
