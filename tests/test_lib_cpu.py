"""CPU-side checks of the product library: it builds, loads and exports every
entry point that include/muca.h declares; host-side validation errors are
reported without touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_1212_3975_amd as pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"\b(muca[A-Z]\w*)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = pm.lib()
    declared = _declared()
    assert "mucaInit" in declared and "mucaSweep" in declared and "mucaReweight" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(pm.EXPORTED) <= set(declared)


def _status(problems, **opt):
    probs = pm.make_problems(problems)
    o = pm.make_options(**opt)
    n = ctypes.c_size_t()
    return pm.lib().mucaWorkspaceSize(probs, len(problems), ctypes.byref(o), ctypes.byref(n)), n.value


class P:
    def __init__(self, model, L, n_chains, seed=1, q=2, beta=0.0):
        self.model, self.L, self.n_chains, self.seed, self.q, self.beta = model, L, n_chains, seed, q, beta


def test_workspace_size_and_validation():
    rc, n = _status([P(0, 64, 4096)])
    assert rc == 0
    # spins + per-chain histograms + production sums dominate
    assert n >= 4096 * 4096 + 12 * 8193 * 4096
    assert _status([P(0, 7, 4)])[0] == -1          # odd L for Ising
    assert _status([P(1, 2, 4, q=8)])[0] == -1     # L < 3
    assert _status([P(1, 8, 4, q=9)])[0] == -1     # q > 8
    assert _status([P(0, 8, 0)])[0] == -1          # no chains
    assert _status([P(3, 8, 4)])[0] == -1          # unknown model
    assert _status([P(2, 8, 4, beta=0.66)])[0] == 0           # multimagnetic Ising
    assert _status([P(2, 7, 4, beta=0.66)])[0] == -1          # odd L
    assert _status([P(2, 8, 4, beta=-0.1)])[0] == -1          # beta < 0
    assert _status([P(2, 8, 4, beta=float("nan"))])[0] == -1  # beta not a number
    assert _status([P(0, 8, 4)], chains_per_wg=12)[0] == 0
    assert _status([P(0, 8, 4)], chains_per_wg=65)[0] == -1
    msg = pm.lib().mucaLastError(None).decode()
    assert "chains_per_wg" in msg
    assert _status([P(0, 8, 4)], chains_per_wg=-1)[0] == -1


def test_init_rejects_small_workspace_without_gpu_calls():
    probs = pm.make_problems([P(0, 8, 4)])
    o = pm.make_options()
    ctx = ctypes.c_void_p()
    rc = pm.lib().mucaInit(ctypes.byref(ctx), probs, 1, ctypes.byref(o), ctypes.c_void_p(256), 16, None)
    assert rc == -2 and not ctx.value
    assert "workspace" in pm.lib().mucaLastError(None).decode()


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    """No fallback: without libmuca.so every entry point of the binding raises."""
    monkeypatch.setattr(pm, "_lib", None)
    monkeypatch.setattr(pm, "LIB_PATH", str(tmp_path / "libmuca.so"))
    with pytest.raises(pm.MucaError, match="missing"):
        pm.lib()
    with pytest.raises(pm.MucaError, match="missing"):
        _status([P(0, 8, 4)])


def test_mlp_workspace_size_and_create_validation_without_gpu_calls():
    """mucaMlpWorkspaceSize accepts 1..2^22 samples and grows with them;
    mucaMlpCreate refuses a small, missing or misaligned workspace before
    any GPU call."""
    L = pm.lib()
    sizes = {}
    for n in (1, 1000, 1 << 22):
        s = ctypes.c_size_t()
        assert L.mucaMlpWorkspaceSize(n, ctypes.byref(s)) == 0
        sizes[n] = s.value
    assert sizes[1] < sizes[1000] < sizes[1 << 22]
    # each sample holds 4 inputs and a target in float32 at least
    assert sizes[1 << 22] - sizes[1] >= ((1 << 22) - 1) * 5 * 4
    for bad in (0, -1, (1 << 22) + 1):
        s = ctypes.c_size_t()
        assert L.mucaMlpWorkspaceSize(bad, ctypes.byref(s)) != 0
        assert "max_samples" in L.mucaMlpLastError(None).decode()
    m = ctypes.c_void_p()
    assert L.mucaMlpCreate(ctypes.byref(m), 1000, 1, ctypes.c_void_p(256), sizes[1000] - 1, None) != 0
    assert not m.value and "workspace" in L.mucaMlpLastError(None).decode()
    assert L.mucaMlpCreate(ctypes.byref(m), 1000, 1, None, sizes[1000], None) != 0
    assert L.mucaMlpCreate(ctypes.byref(m), 1000, 1, ctypes.c_void_p(256 + 16), sizes[1000], None) != 0
    assert "aligned" in L.mucaMlpLastError(None).decode()


def test_static_reweighting_validates_before_touching_a_gpu():
    """mucaReweightStatic refuses bad arguments and sizes beyond its static
    array on the host, before any HIP call (this runs without a GPU)."""
    import numpy as np
    L = 8
    nb = 2 * L * L + 1
    lnW, cnt, sab = np.zeros(nb), np.ones(nb, np.int64), np.zeros(nb, np.int64)
    b = np.array([0.4])
    cases = [
        (dict(model=0, L=7), "even L"),                       # odd Ising L
        (dict(model=0, L=258), "even L"),                     # beyond L = 256
        (dict(model=1, L=257), "Potts needs L"),
        (dict(model=2), "model must be"),
        (dict(betas=np.zeros(4097)), "n_betas"),              # beyond 4096 beta
        (dict(lnW=np.full(nb, np.nan)), "not finite"),
        (dict(cnt=np.zeros(nb, np.int64)), "no production data"),
        (dict(cnt=-np.ones(nb, np.int64)), "negative"),
        (dict(sabs=None), "NULL"),                             # Ising without |M| sums
        (dict(betas=np.array([np.inf])), "not finite"),
    ]
    for kw, msg in cases:
        args = dict(model=0, L=L, lnW=lnW, cnt=cnt, sabs=sab, betas=b)
        args.update(kw)
        with pytest.raises(pm.MucaError, match=msg):
            pm.reweight_static(**args)
    # a size mismatch between the arrays is refused by the binding
    with pytest.raises(ValueError):
        pm.reweight_static(0, L, lnW, cnt[:-1], sab, b)
    # n_bins must be 2N+1 for the stated L
    with pytest.raises(pm.MucaError, match="2N"):
        pm.reweight_static(0, 10, lnW, cnt, sab, b)
