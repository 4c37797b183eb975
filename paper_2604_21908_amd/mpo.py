"""ctypes binding of libmpo (include/mpo.h): argument marshalling only.

Every step of the bond update runs in the HIP kernels of libmpo.so; this
module converts NumPy gate matrices to the C layout and status codes to
exceptions.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpo.so")

FP64, FP32, MIXED = 0, 1, 2
CUT_REL_SV, CUT_WEIGHT = 0, 1
PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}
STATUS = {0: "MPO_OK", 1: "MPO_WARN_NOCONV", -1: "MPO_EINVAL", -2: "MPO_ENOMEM", -3: "MPO_EHIP",
          -4: "MPO_ENUMERIC", -5: "MPO_EOVERFLOW"}
SIDE_NAMES = {0: "L", 1: "R", 2: "B"}

EXPORTED = ["mpo_init_identity", "mpo_absorb_gate_pair", "mpo_absorb_gate_pair_noalloc", "mpo_absorb_batch", "mpo_unswap_sweep",
            "mpo_extract_peak", "mpo_sample", "mpo_free", "mpo_bond_dims", "mpo_total_elements", "mpo_singular_values",
            "mpo_read_site", "mpo_load_state", "mpo_sync", "mpo_copy_state", "mpo_tau_reached", "mpo_trial_swap", "mpo_counters",
            "mpo_profile", "mpo_tuning_report", "mpo_tuning_set", "mpo_last_error", "mpo_version",
            "mpo_group_create", "mpo_group_free", "mpo_group_absorb", "mpo_group_unswap", "mpo_group_profile",
            "mpo_group_last_error"]
COUNTERS = ["updates", "trials", "trials_reused", "commits_undone", "hook_allocs", "graph_replays",
            "graph_captures"]
PROF_CLASSES = ["theta_gemm", "gate", "jacobi_init", "jacobi_gram", "finalize", "writeback", "writeback_gemm", "qr",
                "reorth", "jacobi_evd", "jacobi_rot"]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class MpoConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("chi_max", ctypes.c_int32), ("cutoff", ctypes.c_double),
                ("cutoff_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("jacobi_tol", ctypes.c_double),
                ("tau_elems", ctypes.c_int64), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class UpdateInfo(ctypes.Structure):
    _fields_ = [("chi_new", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("discarded_weight", ctypes.c_double), ("total_weight", ctypes.c_double),
                ("panel_rotations", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class UnswapOpts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("relaxed", ctypes.c_int32), ("max_iters", ctypes.c_int32)]


class SwapEntry(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("bond", ctypes.c_int32)]


class MpoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmpo.so is not built ({path}); run `python -m paper_2604_21908_amd.build`")
    # torch ships its own HIP runtime.  Loaded first, it also serves libmpo's
    # libamdhip64 dependency, so the process holds one runtime and the streams
    # torch hands over are valid in libmpo.  Loaded the other way round, the
    # process would hold two runtimes and torch's streams would be foreign to
    # libmpo.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    lib.mpo_init_identity.argtypes = [ctypes.POINTER(MpoConfig), P, ctypes.POINTER(P)]
    lib.mpo_absorb_gate_pair.argtypes = [P, I32, dp, dp, ctypes.POINTER(UpdateInfo)]
    lib.mpo_absorb_gate_pair_noalloc.argtypes = [P, I32, dp, dp, ctypes.POINTER(UpdateInfo)]
    lib.mpo_absorb_batch.argtypes = [P, I32, ctypes.POINTER(I32), dp, dp, ctypes.POINTER(UpdateInfo)]
    lib.mpo_unswap_sweep.argtypes = [P, ctypes.POINTER(UnswapOpts), ctypes.POINTER(SwapEntry), I32,
                                     ctypes.POINTER(I32)]
    lib.mpo_extract_peak.argtypes = [P, ctypes.POINTER(ctypes.c_uint8), dp, dp]
    lib.mpo_sample.argtypes = [P, I32, dp, ctypes.POINTER(ctypes.c_uint8), dp]
    lib.mpo_free.argtypes = [P]
    lib.mpo_free.restype = None
    lib.mpo_bond_dims.argtypes = [P, ctypes.POINTER(I32)]
    lib.mpo_total_elements.argtypes = [P, ctypes.POINTER(I64)]
    lib.mpo_singular_values.argtypes = [P, I32, dp, I32, ctypes.POINTER(I32)]
    lib.mpo_read_site.argtypes = [P, I32, dp, I64, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.mpo_load_state.argtypes = [P, ctypes.POINTER(I32), dp, dp]
    lib.mpo_sync.argtypes = [P]
    lib.mpo_copy_state.argtypes = [P, P]
    lib.mpo_tau_reached.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I64)]
    lib.mpo_trial_swap.argtypes = [P, I32, I32, ctypes.POINTER(UpdateInfo)]
    lib.mpo_counters.argtypes = [P, ctypes.POINTER(I64), I32]
    lib.mpo_profile.argtypes = [P, I32, dp, ctypes.POINTER(I64)]
    lib.mpo_tuning_report.argtypes = [ctypes.c_char_p, I32]
    lib.mpo_tuning_report.restype = ctypes.c_int32
    lib.mpo_tuning_set.argtypes = [I32]
    lib.mpo_last_error.argtypes = [P]
    lib.mpo_last_error.restype = ctypes.c_char_p
    lib.mpo_version.argtypes = []
    lib.mpo_version.restype = ctypes.c_char_p
    lib.mpo_group_create.argtypes = [I32, P, ctypes.POINTER(P)]
    lib.mpo_group_free.argtypes = [P]
    lib.mpo_group_free.restype = None
    lib.mpo_group_absorb.argtypes = [P, I32, ctypes.POINTER(P), ctypes.POINTER(I32), dp, dp,
                                     ctypes.POINTER(UpdateInfo)]
    lib.mpo_group_unswap.argtypes = [P, I32, ctypes.POINTER(P), ctypes.POINTER(UnswapOpts), ctypes.POINTER(SwapEntry),
                                     I32, ctypes.POINTER(I32)]
    lib.mpo_group_profile.argtypes = [P, I32, dp, ctypes.POINTER(I64)]
    lib.mpo_group_last_error.argtypes = [P]
    lib.mpo_group_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("mpo_free", "mpo_last_error", "mpo_version", "mpo_group_free", "mpo_group_last_error"):
            getattr(lib, name).restype = ctypes.c_int32
    _lib = lib
    return lib


def _gate_ptr(g):
    if g is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(g, dtype=np.complex128).reshape(4, 4)).view(np.float64).reshape(32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class TorchAllocator:
    """alloc/free hooks of mpo_config_t backed by PyTorch's caching allocator
    on one stream; `limit` (bytes) makes allocations beyond it fail, which the
    library reports as MPO_ENOMEM."""

    def __init__(self, stream=None, limit: Optional[int] = None):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        if isinstance(stream, ctypes.c_void_p):
            stream = stream.value
        self.stream = stream          # raw hipStream_t (int) or None: the current stream
        self.limit = limit
        self.live = {}
        self.calls = 0
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        try:
            if self.limit is not None and sum(self.live.values()) + nbytes > self.limit:
                return None
            ptr = self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            self.live[int(ptr)] = int(nbytes)
            self.calls += 1
            return int(ptr)
        except Exception:
            return None

    def _free(self, ptr, _ctx):
        try:
            if ptr and int(ptr) in self.live:
                del self.live[int(ptr)]
                self.torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    @property
    def bytes_live(self) -> int:
        return sum(self.live.values())


class MPO:
    """One device-resident MPO (a libmpo handle).  By default its device
    memory comes from PyTorch's caching allocator (allocator="torch"); pass
    allocator=None for hipMalloc, or a TorchAllocator instance."""

    def __init__(self, n: int, chi_max: int, cutoff: float, cutoff_mode: int = CUT_REL_SV,
                 precision: int = FP64, max_sweeps: int = 0, jacobi_tol: float = 0.0, stream=None,
                 tau_elems: int = 0, allocator="torch"):
        self.lib = load_library()
        self.n = n
        self.precision = precision
        st = stream if stream is not None else _current_stream()
        if allocator == "torch":
            allocator = TorchAllocator(st)
        self.allocator = allocator
        cfg = MpoConfig(n, chi_max, cutoff, cutoff_mode, precision, max_sweeps, jacobi_tol, int(tau_elems))
        if allocator is not None:
            cfg.alloc = allocator.alloc_fn
            cfg.free = allocator.free_fn
        h = ctypes.c_void_p()
        s = self.lib.mpo_init_identity(ctypes.byref(cfg), st, ctypes.byref(h))
        if s != 0:
            raise MpoError(s, "mpo_init_identity failed")
        self.h = h

    # ---------------------------------------------------------------- utils
    def _check(self, s: int, what: str, ok=(0,)):
        if s in ok:
            return s
        msg = self.lib.mpo_last_error(self.h).decode() if self.h else ""
        raise MpoError(s, f"{what}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpo_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- calls
    def absorb(self, bond: int, g_out=None, g_in=None) -> dict:
        ko, po = _gate_ptr(g_out)
        ki, pi = _gate_ptr(g_in)
        info = UpdateInfo()
        s = self.lib.mpo_absorb_gate_pair(self.h, bond, po, pi, ctypes.byref(info))
        self._check(s, "mpo_absorb_gate_pair", ok=(0, 1))
        return dict(k=info.chi_new, sweeps=info.sweeps, discarded=info.discarded_weight,
                    total=info.total_weight, rotations=info.panel_rotations, noconv=(s == 1))

    def absorb_noalloc(self, bond: int, g_out=None, g_in=None) -> dict:
        """mpo_absorb_gate_pair_noalloc: the same update with its workspace
        in the library's static scratch array (no device allocation)."""
        ko, po = _gate_ptr(g_out)
        ki, pi = _gate_ptr(g_in)
        info = UpdateInfo()
        s = self.lib.mpo_absorb_gate_pair_noalloc(self.h, bond, po, pi, ctypes.byref(info))
        self._check(s, "mpo_absorb_gate_pair_noalloc", ok=(0, 1))
        return dict(k=info.chi_new, sweeps=info.sweeps, discarded=info.discarded_weight,
                    total=info.total_weight, rotations=info.panel_rotations, noconv=(s == 1))

    def absorb_batch(self, bonds: Sequence[int], g_outs: Sequence, g_ins: Sequence) -> List[dict]:
        cnt = len(bonds)
        if cnt == 0:
            return []
        b = (ctypes.c_int32 * cnt)(*bonds)
        go = np.zeros((cnt, 32))
        gi = np.zeros((cnt, 32))
        for j in range(cnt):
            if g_outs[j] is not None:
                go[j] = np.ascontiguousarray(np.asarray(g_outs[j], np.complex128)).view(np.float64).reshape(32)
            if g_ins[j] is not None:
                gi[j] = np.ascontiguousarray(np.asarray(g_ins[j], np.complex128)).view(np.float64).reshape(32)
        infos = (UpdateInfo * cnt)()
        dp = ctypes.POINTER(ctypes.c_double)
        s = self.lib.mpo_absorb_batch(self.h, cnt, b, go.ctypes.data_as(dp), gi.ctypes.data_as(dp), infos)
        self._check(s, "mpo_absorb_batch", ok=(0, 1))
        return [dict(k=x.chi_new, sweeps=x.sweeps, discarded=x.discarded_weight, total=x.total_weight,
                     rotations=x.panel_rotations) for x in infos]

    def unswap(self, schedule: str = "parallel", relaxed: bool = False, max_iters: int = 20) -> List[Tuple[str, int]]:
        opts = UnswapOpts(1 if schedule == "parallel" else 0, int(relaxed), max_iters)
        cap = max(64, 4 * max_iters * self.n)
        log = (SwapEntry * cap)()
        nacc = ctypes.c_int32()
        s = self.lib.mpo_unswap_sweep(self.h, ctypes.byref(opts), log, cap, ctypes.byref(nacc))
        self._check(s, "mpo_unswap_sweep", ok=(0, 1))
        return [(SIDE_NAMES[log[j].side], int(log[j].bond)) for j in range(nacc.value)]

    def extract_peak(self) -> Tuple[np.ndarray, float, float]:
        bits = (ctypes.c_uint8 * self.n)()
        p = ctypes.c_double()
        n2 = ctypes.c_double()
        s = self.lib.mpo_extract_peak(self.h, bits, ctypes.byref(p), ctypes.byref(n2))
        self._check(s, "mpo_extract_peak")
        return np.array(bits[:], dtype=np.uint8), p.value, n2.value

    def sample(self, uniforms: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        """mpo_sample: one sample per row of `uniforms` (count x n in [0, 1));
        returns (site bits, count x n; probability of each sampled string)."""
        u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
        if u.ndim != 2 or u.shape[1] != self.n:
            raise ValueError("uniforms must have shape (count, n)")
        cnt = u.shape[0]
        bits = np.zeros((cnt, self.n), dtype=np.uint8)
        probs = np.zeros(cnt)
        dp = ctypes.POINTER(ctypes.c_double)
        s = self.lib.mpo_sample(self.h, cnt, u.ctypes.data_as(dp), bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                probs.ctypes.data_as(dp))
        self._check(s, "mpo_sample")
        return bits, probs

    def bond_dims(self) -> List[int]:
        d = (ctypes.c_int32 * (self.n - 1))()
        self._check(self.lib.mpo_bond_dims(self.h, d), "mpo_bond_dims")
        return list(d)

    def total_elements(self) -> int:
        v = ctypes.c_int64()
        self._check(self.lib.mpo_total_elements(self.h, ctypes.byref(v)), "mpo_total_elements")
        return int(v.value)

    def singular_values(self, bond: int) -> np.ndarray:
        cap = 4096
        out = np.zeros(cap)
        cnt = ctypes.c_int32()
        s = self.lib.mpo_singular_values(self.h, bond, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap,
                                         ctypes.byref(cnt))
        self._check(s, "mpo_singular_values")
        return out[:cnt.value].copy()

    def read_site(self, i: int) -> np.ndarray:
        dims = self.bond_dims()
        cl = 1 if i == 0 else dims[i - 1]
        cr = 1 if i == self.n - 1 else dims[i]
        out = np.zeros(cl * 4 * cr, dtype=np.complex128)
        a, b = ctypes.c_int32(), ctypes.c_int32()
        s = self.lib.mpo_read_site(self.h, i, out.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   2 * out.size, ctypes.byref(a), ctypes.byref(b))
        self._check(s, "mpo_read_site")
        return out.reshape(a.value, 4, b.value)

    def load_state(self, sites: Sequence[np.ndarray], lams: Sequence[np.ndarray]) -> None:
        dims = [int(l.size) for l in lams]
        d = (ctypes.c_int32 * len(dims))(*dims)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(s, np.complex128).reshape(-1) for s in sites]))
        lam = np.ascontiguousarray(np.concatenate([np.asarray(l, np.float64).reshape(-1) for l in lams]))
        dp = ctypes.POINTER(ctypes.c_double)
        s = self.lib.mpo_load_state(self.h, d, flat.view(np.float64).ctypes.data_as(dp), lam.ctypes.data_as(dp))
        self._check(s, "mpo_load_state")

    def sync(self):
        self._check(self.lib.mpo_sync(self.h), "mpo_sync")

    def copy_from(self, other: "MPO") -> None:
        """mpo_copy_state: this MPO becomes an exact copy of `other`."""
        self._check(self.lib.mpo_copy_state(self.h, other.h), "mpo_copy_state")

    def tau_reached(self) -> bool:
        r = ctypes.c_int32()
        self._check(self.lib.mpo_tau_reached(self.h, ctypes.byref(r), None), "mpo_tau_reached")
        return bool(r.value)

    def trial_swap(self, bond: int, side: int) -> dict:
        info = UpdateInfo()
        s = self.lib.mpo_trial_swap(self.h, bond, side, ctypes.byref(info))
        self._check(s, "mpo_trial_swap", ok=(0, 1))
        return dict(k=info.chi_new, sweeps=info.sweeps, discarded=info.discarded_weight,
                    total=info.total_weight, noconv=(s == 1))

    def counters(self) -> dict:
        out = (ctypes.c_int64 * len(COUNTERS))()
        self._check(self.lib.mpo_counters(self.h, out, len(COUNTERS)), "mpo_counters")
        return {c: int(out[i]) for i, c in enumerate(COUNTERS)}

    def profile(self, on: bool) -> dict:
        """Returns {class: (ms, launches)} accumulated so far, resets, and
        switches kernel timing on or off."""
        nc = len(PROF_CLASSES)
        ms = np.zeros(nc)
        cnt = (ctypes.c_int64 * nc)()
        s = self.lib.mpo_profile(self.h, int(on), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cnt)
        self._check(s, "mpo_profile")
        return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(PROF_CLASSES)}


def _pack_gates(gs, cnt):
    out = np.zeros((cnt, 32))
    for j in range(cnt):
        if gs[j] is not None:
            out[j] = np.ascontiguousarray(np.asarray(gs[j], np.complex128)).view(np.float64).reshape(32)
    return out


class Group:
    """Workspace + stream shared by batched updates of several MPOs
    (mpo_group_*): one call applies updates on many handles at once."""

    def __init__(self, precision: int = FP64, stream=None):
        self.lib = load_library()
        g = ctypes.c_void_p()
        st = stream if stream is not None else _current_stream()
        s = self.lib.mpo_group_create(precision, st, ctypes.byref(g))
        if s != 0:
            raise MpoError(s, "mpo_group_create failed")
        self.g = g

    def close(self):
        if getattr(self, "g", None):
            self.lib.mpo_group_free(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def absorb(self, mpos: Sequence["MPO"], bonds: Sequence[int], g_outs: Sequence, g_ins: Sequence) -> List[dict]:
        cnt = len(bonds)
        if cnt == 0:
            return []
        hs = (ctypes.c_void_p * cnt)(*[m.h.value for m in mpos])
        b = (ctypes.c_int32 * cnt)(*bonds)
        go, gi = _pack_gates(g_outs, cnt), _pack_gates(g_ins, cnt)
        infos = (UpdateInfo * cnt)()
        dp = ctypes.POINTER(ctypes.c_double)
        s = self.lib.mpo_group_absorb(self.g, cnt, hs, b, go.ctypes.data_as(dp), gi.ctypes.data_as(dp), infos)
        if s not in (0, 1):
            raise MpoError(s, "mpo_group_absorb: " + self.lib.mpo_group_last_error(self.g).decode())
        return [dict(k=x.chi_new, sweeps=x.sweeps, discarded=x.discarded_weight, total=x.total_weight,
                     rotations=x.panel_rotations) for x in infos]

    def unswap(self, mpos: Sequence["MPO"], relaxed: bool = False, max_iters: int = 20) -> List[List[Tuple[str, int]]]:
        """Parallel unswapping of several MPOs in lockstep (mpo_group_unswap);
        one accepted-swap log per MPO, equal to its lone mpo_unswap_sweep log."""
        cnt = len(mpos)
        if cnt == 0:
            return []
        hs = (ctypes.c_void_p * cnt)(*[m.h.value for m in mpos])
        opts = UnswapOpts(1, int(relaxed), max_iters)
        cap = max(64, 4 * max_iters * max(m.n for m in mpos))
        logs = (SwapEntry * (cap * cnt))()
        nacc = (ctypes.c_int32 * cnt)()
        s = self.lib.mpo_group_unswap(self.g, cnt, hs, ctypes.byref(opts), logs, cap, nacc)
        if s not in (0, 1):
            raise MpoError(s, "mpo_group_unswap: " + self.lib.mpo_group_last_error(self.g).decode())
        return [[(SIDE_NAMES[logs[p * cap + j].side], int(logs[p * cap + j].bond)) for j in range(nacc[p])]
                for p in range(cnt)]

    def profile(self, on: bool) -> dict:
        nc = len(PROF_CLASSES)
        ms = np.zeros(nc)
        cnt = (ctypes.c_int64 * nc)()
        s = self.lib.mpo_group_profile(self.g, int(on), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cnt)
        if s != 0:
            raise MpoError(s, "mpo_group_profile")
        return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(PROF_CLASSES)}


def tuning_report() -> str:
    """The sweep autotuner's table (mpo_tuning_report)."""
    lib = load_library()
    n = lib.mpo_tuning_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib.mpo_tuning_report(buf, n + 1)
    return buf.value.decode()


def tuning_set(mode: int) -> None:
    """mpo_tuning_set: -1 autotuner, -2 fixed defaults, 0..5 one choice."""
    s = load_library().mpo_tuning_set(int(mode))
    if s != 0:
        raise MpoError(s, "mpo_tuning_set")


def version() -> str:
    return load_library().mpo_version().decode()
