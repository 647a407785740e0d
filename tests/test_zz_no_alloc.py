"""nmf_foldin_noalloc (the fold-in entry point whose workspace is the library's
own device array) against nmf_foldin with a caller-allocated workspace: the
same kernels on the same inputs, so the results must be identical.  Two calls
in a row, the second with fewer documents, show that what the first call left
in the shared array does not leak into the second."""
import numpy as np
import pytest

import datagen
from oracle import hals
from tests.gpu_util import EPS, gpu_plan, oracle_A, small_bow, sparse_init

pytestmark = pytest.mark.gpu


def _setup(cuda, K):
    c = small_bow(2000, 900)
    W0, H0 = sparse_init(c, K)
    Ao = oracle_A(c.A)
    W = hals.normalize_columns(W0)
    H = H0.astype(np.float64)
    for _ in range(3):
        W, H = hals.sweep(Ao, W, H, EPS)
    plan = gpu_plan(c.A, W.astype(np.float32), H.astype(np.float32), cuda)
    return c, plan


@pytest.mark.parametrize("K,init", [(16, "given"), (200, "wta"), (40, "mlp")])
def test_foldin_noalloc_matches_foldin(cuda, K, init):
    import torch

    from paper_1904_07935_amd.api import Matrix, Mlp
    c, plan = _setup(cuda, K)
    mlp = Mlp(K, hidden=64, device=cuda, seed=3) if init == "mlp" else None
    for Dn, seed in ((700, 7), (230, 8)):  # the second call is smaller
        new = datagen.bag_of_words_docs(Dn, 1.1, 77.0, seed, c.perm, c.idf)
        M = Matrix.from_csr(new, cuda)
        _, H0 = datagen.uniform_init_matched(c.A.rows, Dn, K, datagen.mean_value(new), seed=4)
        Ha = torch.tensor(np.ascontiguousarray(H0.T), device=cuda)
        Hb = Ha.clone()
        ta = plan.foldin(M, Ha, init=init, mlp=mlp, n_sweeps=12)
        na = plan.foldin_sweeps
        tb = plan.foldin(M, Hb, init=init, mlp=mlp, n_sweeps=12, noalloc=True)
        nb = plan.foldin_sweeps
        torch.cuda.synchronize()
        assert na == nb == 12
        assert torch.equal(Ha, Hb), (Dn, float((Ha - Hb).abs().max()))
        assert ta == tb
        # with a tolerance stop as well
        Hc = torch.tensor(np.ascontiguousarray(H0.T), device=cuda)
        Hd = Hc.clone()
        tc = plan.foldin(M, Hc, init=init, mlp=mlp, n_sweeps=200, tol=1e-6)
        nc = plan.foldin_sweeps
        td = plan.foldin(M, Hd, init=init, mlp=mlp, n_sweeps=200, tol=1e-6, noalloc=True)
        nd = plan.foldin_sweeps
        assert nc == nd and tc == td and torch.equal(Hc, Hd)
    plan.close()


def test_foldin_noalloc_rejects_inputs_beyond_its_array(cuda):
    """More documents than the library's array can hold: NMF_E_WORKSPACE, and
    Ht_new is left untouched."""
    import torch

    from paper_1904_07935_amd._lib import NmfError
    from paper_1904_07935_amd.api import Matrix
    K = 200
    c, plan = _setup(cuda, K)
    Dn = 90000  # R' alone is 72 MB at K = 200
    V = c.A.rows
    new = datagen.Csr(Dn, V, np.arange(Dn + 1, dtype=np.int32),
                      (np.arange(Dn) % V).astype(np.int32), np.ones(Dn, np.float32))
    M = Matrix.from_csr(new, cuda)
    Ht = torch.full((Dn, K), 0.5, device=cuda)
    with pytest.raises(NmfError) as e:
        plan.foldin(M, Ht, init="given", n_sweeps=3, noalloc=True)
    assert e.value.status == -3
    assert torch.all(Ht == 0.5)
    plan.close()
