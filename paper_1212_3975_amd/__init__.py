"""MI355X multicanonical (MUCA) sampling: Python binding of libmuca.so.

Argument marshalling only: every step of the sampling path runs in the HIP
library (include/muca.h).  PyTorch supplies the device workspace and the
stream.  The binding refuses to run without the compiled library.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmuca.so")

ISING, POTTS, ISING_MAG = 0, 1, 2
REC_NONE, REC_MUCA, REC_PROD = 0, 1, 2
GET_H, GET_LNW, GET_T, GET_SPINS, GET_K, GET_M, GET_CHAIN_H, GET_PROD_CNT, GET_PROD_ABSM, GET_SWEEP, GET_REACH = range(11)

EXPORTED = ["mucaWorkspaceSize", "mucaInit", "mucaSetLogWeights", "mucaSweep", "mucaMergeUpdate",
            "mucaIterate", "mucaReweight", "mucaClearProduction", "mucaGet", "mucaLaunchInfo",
            "mucaSweepTiming", "mucaCheckpoint", "mucaRestore", "mucaProblemInfo", "mucaDestroy", "mucaLastError",
            "mucaEqualHeight", "mucaInterfaceTension", "mucaReweightStatic",
            "mucaMlpWorkspaceSize", "mucaMlpCreate", "mucaMlpSetParams", "mucaMlpGetParams", "mucaMlpClearData",
            "mucaMlpAddData", "mucaMlpAddWeights", "mucaMlpNumSamples", "mucaMlpTrain", "mucaMlpGradients",
            "mucaMlpPredict", "mucaMlpSetLogWeights", "mucaMlpDestroy", "mucaMlpLastError"]
MLP_PARAMS = 8705


class MucaError(RuntimeError):
    pass


class Problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("q", ctypes.c_int32), ("L", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("seed", ctypes.c_uint64), ("beta", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("chains_per_wg", ctypes.c_int32), ("rng_mode", ctypes.c_int32),
                ("spin_placement", ctypes.c_int32), ("table_placement", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("production", ctypes.c_int32),
                ("flat_ratio", ctypes.c_double), ("flat_rule", ctypes.c_int32),
                ("tune_sweeps", ctypes.c_int32), ("correction", ctypes.c_int32), ("wait_polls", ctypes.c_int32),
                ("update_norm", ctypes.c_int32), ("pad", ctypes.c_int32)]


class IterStats(ctypes.Structure):
    _fields_ = [("k_lo", ctypes.c_int32), ("k_hi", ctypes.c_int32), ("visited", ctypes.c_int32),
                ("reachable", ctypes.c_int32), ("covered", ctypes.c_int32), ("flat", ctypes.c_int32),
                ("min_over_max", ctypes.c_double), ("min_over_avg", ctypes.c_double),
                ("max_over_avg", ctypes.c_double), ("total", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LaunchInfo(ctypes.Structure):
    _fields_ = [("chains_per_wg", ctypes.c_int32), ("rng_mode", ctypes.c_int32),
                ("spin_placement", ctypes.c_int32), ("table_placement", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("n_workgroups", ctypes.c_int32),
                ("fast_walker", ctypes.c_int32), ("walker", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("pad")}


_lib = None


def lib():
    """Loads libmuca.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MucaError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                            "or python paper_1212_3975_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
        PP = ctypes.POINTER(Problem)
        PO = ctypes.POINTER(Options)
        L.mucaWorkspaceSize.argtypes = [PP, i32, PO, ctypes.POINTER(sz)]
        L.mucaInit.argtypes = [ctypes.POINTER(vp), PP, i32, PO, vp, sz, vp]
        L.mucaSetLogWeights.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), i32]
        L.mucaSweep.argtypes = [vp, i64, i32]
        L.mucaMergeUpdate.argtypes = [vp, i32, ctypes.POINTER(IterStats)]
        L.mucaIterate.argtypes = [vp, i64, ctypes.POINTER(IterStats)]
        L.mucaReweight.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), i32,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
        L.mucaClearProduction.argtypes = [vp]
        L.mucaGet.argtypes = [vp, i32, i32, vp, sz]
        L.mucaLaunchInfo.argtypes = [vp, i32, ctypes.POINTER(LaunchInfo)]
        L.mucaSweepTiming.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
        L.mucaCheckpoint.argtypes = [vp, vp, ctypes.POINTER(sz)]
        L.mucaRestore.argtypes = [vp, vp, sz]
        L.mucaProblemInfo.argtypes = [vp, i32, PP]
        L.mucaDestroy.argtypes = [vp]
        L.mucaDestroy.restype = None
        L.mucaLastError.argtypes = [vp]
        L.mucaLastError.restype = ctypes.c_char_p
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(i32)
        L.mucaEqualHeight.argtypes = [i32, i32, dp, ctypes.POINTER(ctypes.c_int64), i32, ctypes.c_double,
                                      ctypes.c_double, dp, dp, ip, dp]
        L.mucaInterfaceTension.argtypes = [vp, i32, ctypes.c_double, ctypes.c_double, dp, dp, ip, dp]
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.mucaReweightStatic.argtypes = [i32, i32, dp, i64p, i64p, i32, dp, i32, dp, dp, dp, vp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.mucaMlpWorkspaceSize.argtypes = [i32, ctypes.POINTER(sz)]
        L.mucaMlpCreate.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_uint64, vp, sz, vp]
        L.mucaMlpSetParams.argtypes = [vp, fp]
        L.mucaMlpGetParams.argtypes = [vp, fp]
        L.mucaMlpClearData.argtypes = [vp]
        L.mucaMlpAddData.argtypes = [vp, fp, fp, i32]
        L.mucaMlpAddWeights.argtypes = [vp, vp, i32]
        L.mucaMlpNumSamples.argtypes = [vp, ctypes.POINTER(i32)]
        L.mucaMlpTrain.argtypes = [vp, i32, ctypes.c_float, fp]
        L.mucaMlpGradients.argtypes = [vp, fp, fp]
        L.mucaMlpPredict.argtypes = [vp, fp, i32, fp]
        L.mucaMlpSetLogWeights.argtypes = [vp, vp, i32]
        L.mucaMlpDestroy.argtypes = [vp]
        L.mucaMlpDestroy.restype = None
        L.mucaMlpLastError.argtypes = [vp]
        L.mucaMlpLastError.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("mucaDestroy", "mucaLastError", "mucaMlpDestroy", "mucaMlpLastError"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != 0:
        msg = lib().mucaLastError(ctx)
        raise MucaError(f"muca error {rc}: {msg.decode() if msg else ''}")


def _dptr(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def make_problems(problems) -> "ctypes.Array":
    arr = (Problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = Problem(int(p.model), int(getattr(p, "q", 2)), int(p.L), int(p.n_chains), int(p.seed),
                         float(getattr(p, "beta", 0.0)))
    return arr


def make_options(**kw) -> Options:
    o = Options()
    o.production = 1
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Muca:
    """One library context: problems, device workspace (a torch tensor) and stream."""

    def __init__(self, problems: Sequence, device: str = "cuda:0", stream=None, **options):
        import torch
        self._torch = torch
        self.problems = list(problems)
        self._probs = make_problems(self.problems)
        self._opts = make_options(**options)
        n = len(self.problems)
        size = ctypes.c_size_t()
        _check(lib().mucaWorkspaceSize(self._probs, n, ctypes.byref(self._opts), ctypes.byref(size)))
        self.workspace = torch.empty(max(size.value, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        self._ctx = ctypes.c_void_p()
        _check(lib().mucaInit(ctypes.byref(self._ctx), self._probs, n, ctypes.byref(self._opts),
                              ctypes.c_void_p(self.workspace.data_ptr()), size.value,
                              ctypes.c_void_p(self.stream.cuda_stream)))

    # -- lifecycle
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().mucaDestroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _c(self, rc):
        _check(rc, self._ctx)

    # -- sampling
    def sweep(self, n_sweeps: int, record: int = REC_NONE):
        self._c(lib().mucaSweep(self._ctx, int(n_sweeps), int(record)))

    def merge_update(self, update: bool = True):
        st = (IterStats * len(self.problems))()
        self._c(lib().mucaMergeUpdate(self._ctx, int(update), st))
        return [s.as_dict() for s in st]

    def iterate(self, n_sweeps: int):
        st = (IterStats * len(self.problems))()
        self._c(lib().mucaIterate(self._ctx, int(n_sweeps), st))
        return [s.as_dict() for s in st]

    def set_log_weights(self, prob: int, lnW: np.ndarray):
        a = np.ascontiguousarray(lnW, np.float64)
        self._c(lib().mucaSetLogWeights(self._ctx, prob, _dptr(a, ctypes.c_double), a.size))

    def clear_production(self):
        self._c(lib().mucaClearProduction(self._ctx))

    def reweight(self, prob: int, betas: Sequence[float]):
        b = np.ascontiguousarray(betas, np.float64)
        e, c, m = (np.zeros(b.size) for _ in range(3))
        self._c(lib().mucaReweight(self._ctx, prob, _dptr(b, ctypes.c_double), b.size,
                                   _dptr(e, ctypes.c_double), _dptr(c, ctypes.c_double),
                                   _dptr(m, ctypes.c_double)))
        return e, c, m

    def interface_tension(self, prob: int, beta_lo: float, beta_hi: float):
        """Equal-height inverse temperature and sigma_od = ln(P_max/P_min)/(2L)
        of problem prob's production data (Sec. 5, Eq. 9)."""
        beta, sigma = ctypes.c_double(), ctypes.c_double()
        k3 = (ctypes.c_int32 * 3)()
        lnP = np.zeros(self._dims(prob)[1])
        self._c(lib().mucaInterfaceTension(self._ctx, prob, float(beta_lo), float(beta_hi), ctypes.byref(beta),
                                           ctypes.byref(sigma), k3, _dptr(lnP, ctypes.c_double)))
        return {"beta": beta.value, "sigma": sigma.value, "k_peaks": tuple(k3), "lnP": lnP}

    # -- state
    def _get(self, what: int, prob: int, dtype, shape):
        out = np.zeros(shape, dtype)
        self._c(lib().mucaGet(self._ctx, what, prob, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def _dims(self, prob):
        p = self.problems[prob]
        N = p.L * p.L
        # bins: k = 0..2N, or m = 0..N up spins for the multimagnetic ensemble
        return N, (N + 1 if p.model == ISING_MAG else 2 * N + 1), p.n_chains

    def H(self, prob=0):
        return self._get(GET_H, prob, np.int64, self._dims(prob)[1])

    def lnW(self, prob=0):
        return self._get(GET_LNW, prob, np.float64, self._dims(prob)[1])

    def table(self, prob=0):
        """The device acceptance table: Ising [N+1][5] (row k/2, column
        dk/2 + 2), Potts [2N+1][9] (row k, column dk + 4), multimagnetic
        [N+1][10] (row m, column j + 5u)."""
        p = self.problems[prob]
        N = p.L * p.L
        shape = {ISING: (N + 1, 5), POTTS: (2 * N + 1, 9), ISING_MAG: (N + 1, 10)}[p.model]
        return self._get(GET_T, prob, np.uint32, shape)

    def spins(self, prob=0):
        """Spins as [C][N] (chain-major) for comparison; the device keeps [N][C]."""
        N, _, C = self._dims(prob)
        return self._get(GET_SPINS, prob, np.uint8, (N, C)).T.copy()

    def k(self, prob=0):
        return self._get(GET_K, prob, np.int32, self._dims(prob)[2])

    def m(self, prob=0):
        return self._get(GET_M, prob, np.int32, self._dims(prob)[2])

    def chain_hist(self, prob=0):
        """Per-chain histograms as [C][2N+1]."""
        N, nb, C = self._dims(prob)
        return self._get(GET_CHAIN_H, prob, np.int32, (nb, C)).T.copy()

    def prod_counts(self, prob=0):
        return self._get(GET_PROD_CNT, prob, np.int64, self._dims(prob)[1])

    def prod_absm(self, prob=0):
        return self._get(GET_PROD_ABSM, prob, np.int64, self._dims(prob)[1])

    def sweep_count(self):
        return int(self._get(GET_SWEEP, 0, np.uint32, 1)[0])

    def reachable(self, prob=0):
        return self._get(GET_REACH, prob, np.uint8, self._dims(prob)[1]).astype(bool)

    def launch_info(self, prob=0):
        li = LaunchInfo()
        self._c(lib().mucaLaunchInfo(self._ctx, prob, ctypes.byref(li)))
        return li.as_dict()

    def sweep_timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int32()
        self._c(lib().mucaSweepTiming(self._ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def checkpoint(self) -> bytes:
        n = ctypes.c_size_t()
        self._c(lib().mucaCheckpoint(self._ctx, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._c(lib().mucaCheckpoint(self._ctx, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)))
        return buf.raw

    def restore(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._c(lib().mucaRestore(self._ctx, ctypes.cast(buf, ctypes.c_void_p), len(blob)))


def _check_mlp(rc, m=None):
    if rc != 0:
        msg = lib().mucaMlpLastError(m)
        raise MucaError(f"muca mlp error {rc}: {msg.decode() if msg else ''}")


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def equal_height(model: int, L: int, lnW, cnt, beta_lo: float, beta_hi: float):
    """mucaEqualHeight on host arrays (no GPU needed): the equal-height inverse
    temperature of the reweighted energy histogram and sigma_od (Sec. 5, Eq. 9)."""
    w = np.ascontiguousarray(lnW, np.float64)
    c = np.ascontiguousarray(cnt, np.int64)
    if w.shape != c.shape:
        raise ValueError("lnW and cnt differ in size")
    beta, sigma = ctypes.c_double(), ctypes.c_double()
    k3 = (ctypes.c_int32 * 3)()
    lnP = np.zeros(w.size)
    rc = lib().mucaEqualHeight(int(model), int(L), _dptr(w, ctypes.c_double),
                               c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), w.size, float(beta_lo),
                               float(beta_hi), ctypes.byref(beta), ctypes.byref(sigma), k3,
                               _dptr(lnP, ctypes.c_double))
    _check(rc)
    return {"beta": beta.value, "sigma": sigma.value, "k_peaks": tuple(k3), "lnP": lnP}


def reweight_static(model: int, L: int, lnW, cnt, sabs, betas, stream=None):
    """mucaReweightStatic: Eq. (2) reweighting of caller-held production data
    (merged counts, |M| sums, log-weights) with no context and no device
    allocation.  Returns (<E>/N, C_V, <|M|>/N) as float64 arrays."""
    w = np.ascontiguousarray(lnW, np.float64)
    c = np.ascontiguousarray(cnt, np.int64)
    a = None if sabs is None else np.ascontiguousarray(sabs, np.int64)
    b = np.ascontiguousarray(betas, np.float64)
    if c.size != w.size or (a is not None and a.size != w.size):
        raise ValueError("lnW, cnt and sabs differ in size")
    e, cv, m = (np.zeros(b.size) for _ in range(3))
    i64 = ctypes.POINTER(ctypes.c_int64)
    sp = None
    if stream is not None:
        sp = ctypes.c_void_p(stream.cuda_stream)
    rc = lib().mucaReweightStatic(int(model), int(L), _dptr(w, ctypes.c_double), c.ctypes.data_as(i64),
                                  None if a is None else a.ctypes.data_as(i64), w.size, _dptr(b, ctypes.c_double),
                                  b.size, _dptr(e, ctypes.c_double), _dptr(cv, ctypes.c_double),
                                  _dptr(m, ctypes.c_double), sp)
    _check(rc)
    return e, cv, m


class Mlp:
    """The learned-initial-weights network (see include/muca.h)."""

    def __init__(self, max_samples: int = 65536, seed: int = 1, device: str = "cuda:0", stream=None):
        import torch
        size = ctypes.c_size_t()
        _check_mlp(lib().mucaMlpWorkspaceSize(int(max_samples), ctypes.byref(size)))
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        self._m = ctypes.c_void_p()
        _check_mlp(lib().mucaMlpCreate(ctypes.byref(self._m), int(max_samples), int(seed),
                                       ctypes.c_void_p(self.workspace.data_ptr()), size.value,
                                       ctypes.c_void_p(self.stream.cuda_stream)))

    def _c(self, rc):
        _check_mlp(rc, self._m)

    def close(self):
        if getattr(self, "_m", None) and self._m.value:
            lib().mucaMlpDestroy(self._m)
            self._m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_params(self, p):
        a = _f32(p)
        assert a.size == MLP_PARAMS
        self._c(lib().mucaMlpSetParams(self._m, _dptr(a, ctypes.c_float)))

    def params(self):
        out = np.zeros(MLP_PARAMS, np.float32)
        self._c(lib().mucaMlpGetParams(self._m, _dptr(out, ctypes.c_float)))
        return out

    def clear_data(self):
        self._c(lib().mucaMlpClearData(self._m))

    def add_data(self, x, y):
        x = _f32(x)
        y = _f32(y)
        self._c(lib().mucaMlpAddData(self._m, _dptr(x, ctypes.c_float), _dptr(y, ctypes.c_float), y.size))

    def add_weights(self, ctx: "Muca", prob: int = 0):
        self._c(lib().mucaMlpAddWeights(self._m, ctx._ctx, prob))

    def num_samples(self):
        n = ctypes.c_int32()
        self._c(lib().mucaMlpNumSamples(self._m, ctypes.byref(n)))
        return n.value

    def train(self, steps: int, lr: float):
        losses = np.zeros(max(steps, 1), np.float32)
        self._c(lib().mucaMlpTrain(self._m, int(steps), float(lr), _dptr(losses, ctypes.c_float)))
        return losses[:steps]

    def gradients(self):
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        self._c(lib().mucaMlpGradients(self._m, _dptr(g, ctypes.c_float), _dptr(loss, ctypes.c_float)))
        return float(loss[0]), g

    def predict(self, x):
        x = _f32(x)
        n = x.size // 4
        y = np.zeros(n, np.float32)
        self._c(lib().mucaMlpPredict(self._m, _dptr(x, ctypes.c_float), n, _dptr(y, ctypes.c_float)))
        return y

    def set_log_weights(self, ctx: "Muca", prob: int = 0):
        self._c(lib().mucaMlpSetLogWeights(self._m, ctx._ctx, prob))
