"""Guard for the oracle pins: plausible slips planted into a copy of the
oracle (on the CPU, in a temporary directory) must each make the pin suite
fail.  The real oracle is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "R sign": ("H[k, :] + R[:, k] - H.T @ S[:, k]", "H[k, :] - R[:, k] - H.T @ S[:, k]"),
    "S row instead of column": ("H.T @ S[:, k]", "H.T @ S[k, :] * 1.0001"),
    "drop Q_kk": ("W[:, k] * Q[k, k] + P[:, k]", "W[:, k] + P[:, k]"),
    "no normalisation": ("W[:, k] = W[:, k] / np.linalg.norm(W[:, k])", "W[:, k] = W[:, k]"),
    "clip at 0": ("np.maximum(eps, W[:, k] * Q[k, k]", "np.maximum(0.0, W[:, k] * Q[k, k]"),
    "P columns permuted": ("P = np.asarray(A @ H.T)", "P = np.asarray(A @ H.T)[:, ::-1]"),
    "phase 1 dropped": ("W_new[:, :a] -= W_old[:, a:b] @ Q[a:b, :a]", "pass"),
    "phase 2 old/new swapped": ("s = W_new[:, a:t] @ Q[t, a:t] + W_old[:, t:b] @ Q[t, t:b]",
                                "s = W_old[:, a:t] @ Q[t, a:t] + W_old[:, t:b] @ Q[t, t:b]"),
    "ragged tile dropped": ("return [(s, min(s + T, K)) for s in range(0, K, T)]",
                            "return [(s, s + T) for s in range(0, K - K % T, T)]"),
    "identity cross term": ("a2 - 2.0 * float(np.sum(W * P))", "a2 - 1.0 * float(np.sum(W * P))"),
    "fold-in Gram scaled": ("S = W.T @ W\n    H = _f64(H0)", "S = W.T @ W * 1.001\n    H = _f64(H0)"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_slip_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "hals.py")).read()
    a, b = MUTATIONS[name]
    assert a in src, "mutation anchor vanished: update the guard"
    for d in ("oracle", "datagen"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d)
    os.makedirs(tmp_path / "tests")
    for f in ("conftest.py", "test_oracle_hals.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tmp_path / "tests" / f)
    (tmp_path / "oracle" / "hals.py").write_text(src.replace(a, b, 1))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle_hals.py"], cwd=tmp_path, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0, f"slip '{name}' passed every pin"


MU_MUTATIONS = {
    "MU H quotient inverted": ("return H * num / ((W.T @ W) @ H + delta)",
                               "return H * ((W.T @ W) @ H + delta) / num"),
    "MU W rule with the old factor dropped": ("return W * num / (W @ (H @ H.T) + delta)",
                                              "return num / (W @ (H @ H.T) + delta)"),
    "MU W rule with H^T H": ("W @ (H @ H.T) + delta", "W @ (H @ H.T) * 1.01 + delta"),
    "MU W rule with the old H": ("    W = mu_w(A, W, H, delta)\n", "    W = mu_w(A, W, H0, delta)\n"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MU_MUTATIONS))
def test_planted_mu_slip_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "mu.py")).read()
    a, b = MU_MUTATIONS[name]
    assert a in src, "mutation anchor vanished: update the guard"
    for d in ("oracle", "datagen"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d)
    os.makedirs(tmp_path / "tests")
    for f in ("conftest.py", "test_oracle_mu.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tmp_path / "tests" / f)
    mutated = src.replace(a, b, 1)
    if "H0" in b:  # keep the sweep's original H in reach
        mutated = mutated.replace("    H = mu_h(A, W, H, delta)\n", "    H0 = H\n    H = mu_h(A, W, H, delta)\n")
    (tmp_path / "oracle" / "mu.py").write_text(mutated)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle_mu.py"], cwd=tmp_path, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0, f"slip '{name}' passed every pin"
