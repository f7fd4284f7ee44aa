"""ctypes binding of libstn.so (include/stn.h): argument marshalling only.

Every step of the ensemble path (sampling, contraction, reduction) runs in the
library's HIP kernels; this module converts a ``workloads.Problem`` into the
C structures, passes PyTorch's caching allocator and current stream to the
library, and copies results back.  There is no fallback: if the library is
missing or the device is unavailable the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# STN_LIBRARY names another build of the same library (e.g. the host-sanitizer build)
LIB_PATH = os.environ.get("STN_LIBRARY") or os.path.join(_HERE, "libstn.so")

GATE_KIND = {"h": 0, "x": 1, "y": 2, "z": 3, "rx": 4, "ry": 5, "rz": 6, "zz": 7, "cx": 8, "u1": 9, "u2": 10}
CHANNEL_KIND = {"bitflip": 0, "depol1": 1, "depol2": 2, "ampdamp": 3, "kraus": 4}

OUT_RHO, OUT_DIAG, OUT_ENERGY, OUT_STATES = 1, 2, 4, 8
PLAN_AUTO, PLAN_SV_LDS, PLAN_SV_TILED, PLAN_LIGHTCONE, PLAN_SV_GATES = 0, 1, 2, 3, 4
PLAN_NAMES = {0: "auto", 1: "sv_lds", 2: "sv_tiled", 3: "lightcone", 4: "sv_gates"}
STATUS = {0: "OK", 1: "INVALID", 2: "UNSUPPORTED", 3: "OOM", 4: "DEVICE", 5: "STATE"}


class StnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"stn {STATUS.get(status, status)}: {msg}")
        self.status = status


class Gate(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("q0", C.c_uint32), ("q1", C.c_uint32), ("theta", C.c_double),
                ("mat", C.POINTER(C.c_double))]


class Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_uint32), ("n_gates", C.c_uint32), ("gates", C.POINTER(Gate))]


class Channel(C.Structure):
    _fields_ = [("after_gate", C.c_uint32), ("kind", C.c_uint32), ("n_qubits", C.c_uint32), ("q0", C.c_uint32),
                ("q1", C.c_uint32), ("param", C.c_double), ("n_kraus", C.c_uint32),
                ("kraus", C.POINTER(C.c_double))]


class NoiseModel(C.Structure):
    _fields_ = [("n_channels", C.c_uint32), ("channels", C.POINTER(Channel))]


class Observable(C.Structure):
    _fields_ = [("n_terms", C.c_uint32), ("uv", C.POINTER(C.c_uint32)), ("w", C.POINTER(C.c_double))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TermNetwork(C.Structure):
    _fields_ = [("term", C.c_uint32), ("u", C.c_uint32), ("v", C.c_uint32), ("n_vars", C.c_uint32),
                ("n_tensors", C.c_uint32), ("tensor_offsets", C.POINTER(C.c_uint32)),
                ("tensor_vars", C.POINTER(C.c_uint32))]


ORDER_FN = C.CFUNCTYPE(C.c_int, C.POINTER(TermNetwork), C.POINTER(C.c_uint32), C.c_void_p)


def _order_callback(fn):
    """Wraps fn(net) -> sequence of variables (net: dict with term, u, v,
    n_vars, tensors = list of variable lists) as an stn_order_fn."""
    def cb(netp, order, _ctx):
        try:
            net = netp.contents
            off = [net.tensor_offsets[i] for i in range(net.n_tensors + 1)]
            tensors = [[net.tensor_vars[j] for j in range(off[t], off[t + 1])] for t in range(net.n_tensors)]
            got = list(fn({"term": net.term, "u": net.u, "v": net.v, "n_vars": net.n_vars, "tensors": tensors}))
            if len(got) != net.n_vars:
                return 1
            for i, x in enumerate(got):
                order[i] = int(x)
            return 0
        except Exception:
            return 1
    return ORDER_FN(cb)


class PlanOpts(C.Structure):
    _fields_ = [("precision", C.c_uint32), ("outputs", C.c_uint32), ("plan_kind", C.c_uint32),
                ("max_batch", C.c_uint32), ("hbm_budget", C.c_uint64), ("order_restarts", C.c_uint32),
                ("order_seed", C.c_uint64), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_ctx", C.c_void_p), ("lc_max_rank", C.c_uint32), ("lc_slice_bits", C.c_uint32),
                ("lc_order_fn", ORDER_FN), ("lc_order_ctx", C.c_void_p), ("sv_full_state", C.c_uint32),
                ("sv_tile_bits", C.c_uint32)]


class PlanStats(C.Structure):
    _fields_ = [("plan_kind", C.c_uint32), ("n_qubits", C.c_uint32), ("n_gates", C.c_uint32),
                ("n_sites", C.c_uint32), ("max_batch", C.c_uint32), ("width", C.c_uint32),
                ("n_passes", C.c_uint32), ("n_steps", C.c_uint32), ("bytes_per_traj", C.c_double),
                ("flops_per_traj", C.c_double), ("peak_bytes", C.c_double), ("lc_width", C.c_uint32),
                ("lc_flops_per_traj", C.c_double), ("variant", C.c_uint32), ("tuned", C.c_uint32),
                ("graphs", C.c_uint32), ("graph_captures", C.c_uint64), ("graph_replays", C.c_uint64),
                ("lc_slices", C.c_uint32), ("lc_slice_bits", C.c_uint32), ("est_s_per_traj", C.c_double),
                ("lc_group", C.c_uint32), ("lc_width_lower_bound", C.c_uint32), ("half_state", C.c_uint32),
                ("tile_bits", C.c_uint32)]


class TuneResult(C.Structure):
    _fields_ = [("n_variants", C.c_uint32), ("chosen", C.c_uint32), ("ms", C.c_double * 8)]


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double)]


KERNEL_NAMES = ["sample", "frame", "sv_lds", "sv_pass", "tile_sum", "herk", "diag", "tn_step"]


class Result(C.Structure):
    _fields_ = [("k_done", C.c_uint64), ("energy_mean", C.c_double), ("energy_se", C.c_double),
                ("trace_mean", C.c_double), ("rho", C.POINTER(C.c_double)), ("diag", C.POINTER(C.c_double)),
                ("energies", C.POINTER(C.c_double))]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("job_share", C.c_double), ("n_streams", C.c_uint32),
                ("max_active", C.c_uint32), ("plan_cache", C.c_uint32), ("precision", C.c_uint32),
                ("chunk_max", C.c_uint32), ("drain_on_destroy", C.c_uint32), ("reserve_cus", C.c_uint32),
                ("graphs", C.c_uint32), ("gang", C.c_uint32)]


class JobResult(C.Structure):
    _fields_ = [("job_id", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_uint32), ("plan_kind", C.c_uint32),
                ("width", C.c_uint32), ("chunk", C.c_uint32), ("K", C.c_uint64), ("k_done", C.c_uint64),
                ("chunks", C.c_uint64), ("energy_mean", C.c_double), ("energy_se", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("error", C.c_char * 96)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("active", C.c_uint64), ("waiting", C.c_uint64), ("trajectories", C.c_uint64),
                ("chunks", C.c_uint64), ("max_active_jobs", C.c_uint64), ("plan_cache_hits", C.c_uint64),
                ("plan_cache_misses", C.c_uint64), ("plans_cached", C.c_uint64), ("autotuned", C.c_uint64),
                ("bytes_in_use", C.c_uint64),
                ("bytes_cached", C.c_uint64), ("bytes_peak", C.c_uint64), ("clock", C.c_double),
                ("gang_launches", C.c_uint64), ("gang_chunks", C.c_uint64)]


EXPORTS = {
    "stn_version": (C.c_char_p, []),
    "stn_last_error": (C.c_char_p, []),
    "stn_plan_opts_default": (None, [C.POINTER(PlanOpts)]),
    "stn_plan_create": (C.c_int, [C.POINTER(Circuit), C.POINTER(NoiseModel), C.POINTER(Observable),
                                  C.POINTER(PlanOpts), C.POINTER(C.c_void_p)]),
    "stn_plan_info": (C.c_int, [C.c_void_p, C.POINTER(PlanStats)]),
    "stn_plan_destroy": (None, [C.c_void_p]),
    "stn_plan_site": (C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.c_uint32]),
    "stn_sample": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32, C.POINTER(C.c_void_p), C.c_void_p]),
    "stn_batch_from_indices": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint8), C.c_uint64, C.c_uint32,
                                         C.POINTER(C.c_void_p), C.c_void_p]),
    "stn_batch_indices": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint8)]),
    "stn_contract": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "stn_batch_results": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "stn_plan_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(TuneResult), C.c_void_p]),
    "stn_plan_set_variant": (C.c_int, [C.c_void_p, C.c_uint32]),
    "stn_plan_set_graphs": (C.c_int, [C.c_void_p, C.c_uint32]),
    "stn_contract_many": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_uint32, C.c_void_p]),
    "stn_contract_dedup": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32), C.c_void_p]),
    "stn_resample": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_void_p]),
    "stn_batch_size": (C.c_uint32, [C.c_void_p]),
    "stn_batch_destroy": (None, [C.c_void_p]),
    "stn_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "stn_profile_read": (C.c_int, [C.c_void_p, C.POINTER(KernelStats)]),
    "stn_accum_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "stn_reduce": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "stn_accum_read": (C.c_int, [C.c_void_p, C.POINTER(Result), C.c_void_p]),
    "stn_accum_destroy": (None, [C.c_void_p]),
    "stn_accum_sample": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "stn_accum_sample_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "stn_server_opts_default": (None, [C.POINTER(ServerOpts)]),
    "stn_server_create": (C.c_int, [C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]),
    "stn_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Circuit), C.POINTER(NoiseModel), C.POINTER(Observable),
                                    C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64)]),
    "stn_server_poll": (C.c_int, [C.c_void_p, C.POINTER(JobResult), C.c_uint32, C.POINTER(C.c_uint32), C.c_double]),
    "stn_server_drain": (C.c_int, [C.c_void_p, C.c_double]),
    "stn_server_stats_read": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "stn_server_clock": (C.c_double, [C.c_void_p]),
    "stn_server_last_error": (C.c_char_p, []),
    "stn_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def load(path: Optional[str] = None):
    """Loads libstn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not built: run python -m paper_2210_15874_amd.build")
    lib = C.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(st):
    if st != 0:
        raise StnError(st, _lib.stn_last_error().decode())


def current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class _TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
        except Exception:  # out of memory: the library reports STN_E_OOM
            return None

    def _free(self, ptr, ctx):
        cuda = getattr(self.torch, "cuda", None)
        if cuda is None:   # interpreter shutdown: torch is torn down already; the process releases the memory
            return
        cuda.caching_allocator_delete(ptr)


def _problem_structs(problem, with_observable):
    gates = (Gate * max(1, len(problem.gates)))()
    keep = []
    for i, g in enumerate(problem.gates):
        gates[i].kind = GATE_KIND[g.kind]
        gates[i].q0 = g.qubits[0]
        gates[i].q1 = g.qubits[1] if len(g.qubits) > 1 else 0
        gates[i].theta = float(g.theta)
        if g.matrix is not None:
            m = np.ascontiguousarray(np.array(g.matrix, dtype=np.complex128).view(np.float64))
            keep.append(m)
            gates[i].mat = m.ctypes.data_as(C.POINTER(C.c_double))
    circ = Circuit(problem.n_qubits, len(problem.gates), gates)
    chans = (Channel * max(1, len(problem.channels)))()
    for i, ch in enumerate(problem.channels):
        chans[i].after_gate = ch.after_gate
        chans[i].kind = CHANNEL_KIND[ch.kind]
        chans[i].n_qubits = len(ch.qubits)
        chans[i].q0 = ch.qubits[0]
        chans[i].q1 = ch.qubits[1] if len(ch.qubits) > 1 else 0
        chans[i].param = float(ch.param)
        if ch.kraus is not None:
            m = np.ascontiguousarray(np.array(ch.kraus, dtype=np.complex128).reshape(-1).view(np.float64))
            keep.append(m)
            chans[i].n_kraus = len(ch.kraus)
            chans[i].kraus = m.ctypes.data_as(C.POINTER(C.c_double))
    noise = NoiseModel(len(problem.channels), chans)
    obs = None
    if with_observable:
        uv = np.ascontiguousarray(np.array(problem.edges, dtype=np.uint32).reshape(-1))
        w = np.ascontiguousarray(np.array(problem.weights, dtype=np.float64))
        keep += [uv, w]
        obs = Observable(len(problem.edges), uv.ctypes.data_as(C.POINTER(C.c_uint32)),
                         w.ctypes.data_as(C.POINTER(C.c_double)))
    return circ, noise, obs, (gates, chans, keep)


class Plan:
    """stn_plan_create for a workloads.Problem."""

    def __init__(self, problem, outputs=OUT_ENERGY, precision=64, plan_kind=PLAN_AUTO, max_batch=0,
                 hbm_budget=0, torch_allocator=True, device=0, lc_max_rank=0, lc_slice_bits=0, lc_order=None,
                 full_state=False, tile_bits=0):
        self.lib = load()
        self.problem = problem
        self.n = problem.n_qubits
        self.S = len(problem.channels)
        self.outputs = outputs
        self.precision = precision
        opts = PlanOpts()
        self.lib.stn_plan_opts_default(C.byref(opts))
        opts.precision = precision
        opts.outputs = outputs
        opts.plan_kind = plan_kind
        opts.max_batch = max_batch
        opts.hbm_budget = hbm_budget
        opts.lc_max_rank = lc_max_rank
        opts.lc_slice_bits = lc_slice_bits
        opts.sv_full_state = 1 if full_state else 0
        opts.sv_tile_bits = tile_bits
        self._order_cb = None
        if lc_order is not None:
            self._order_cb = _order_callback(lc_order)
            opts.lc_order_fn = self._order_cb
        self._alloc = None
        if torch_allocator:
            self._alloc = _TorchAllocator(device)
            opts.dev_alloc = self._alloc.alloc
            opts.dev_free = self._alloc.free
        circ, noise, obs, self._keep = _problem_structs(problem, bool(outputs & OUT_ENERGY))
        h = C.c_void_p()
        _check(self.lib.stn_plan_create(C.byref(circ), C.byref(noise), C.byref(obs) if obs else None,
                                        C.byref(opts), C.byref(h)))
        self.h = h

    def info(self):
        s = PlanStats()
        _check(self.lib.stn_plan_info(self.h, C.byref(s)))
        d = {f: getattr(s, f) for f, _ in PlanStats._fields_}
        d["plan_name"] = PLAN_NAMES.get(d["plan_kind"], "?")
        return d

    def site_thresholds(self, s):
        J = C.c_uint32()
        T = (C.c_uint64 * 16)()
        _check(self.lib.stn_plan_site(self.h, s, C.byref(J), T, 16))
        return [int(T[j]) for j in range(J.value)]

    def sample(self, seed, k0, K, stream=None):
        h = C.c_void_p()
        _check(self.lib.stn_sample(self.h, int(seed), int(k0), int(K), C.byref(h),
                                   stream if stream is not None else current_stream()))
        return Batch(self, h, K)

    def batch_from_indices(self, idx, k0=0, stream=None):
        idx = np.ascontiguousarray(idx, dtype=np.uint8)
        K = idx.shape[0]
        assert idx.shape == (K, self.S)
        h = C.c_void_p()
        _check(self.lib.stn_batch_from_indices(self.h, idx.ctypes.data_as(C.POINTER(C.c_uint8)), int(k0), K,
                                               C.byref(h), stream if stream is not None else current_stream()))
        return Batch(self, h, K)

    def contract(self, batch, stream=None):
        _check(self.lib.stn_contract(self.h, batch.h, stream if stream is not None else current_stream()))

    def contract_dedup(self, batch, stream=None):
        """Contracts each distinct trajectory once; returns their number."""
        u = C.c_uint32()
        _check(self.lib.stn_contract_dedup(self.h, batch.h, C.byref(u),
                                           stream if stream is not None else current_stream()))
        return u.value

    def autotune(self, batch, reps=2, stream=None):
        """Times every launch shape of this plan's contraction on `batch` and
        keeps the fastest; returns {"chosen": v, "ms": [...]}."""
        r = TuneResult()
        _check(self.lib.stn_plan_autotune(self.h, batch.h, int(reps), C.byref(r),
                                          stream if stream is not None else current_stream()))
        return {"chosen": r.chosen, "ms": [r.ms[i] for i in range(r.n_variants)]}

    def set_variant(self, v):
        _check(self.lib.stn_plan_set_variant(self.h, int(v)))

    def set_graphs(self, on=True):
        """Contractions of a reused batch replay a captured HIP graph."""
        _check(self.lib.stn_plan_set_graphs(self.h, 1 if on else 0))

    def resample(self, batch, seed, k0, K, stream=None):
        """Refills `batch` with trajectories k0 .. k0+K-1 (buffers reused)."""
        _check(self.lib.stn_resample(batch.h, int(seed), int(k0), int(K),
                                     stream if stream is not None else current_stream()))
        batch.K = int(K)
        return batch

    def profile(self, enable=True):
        _check(self.lib.stn_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        arr = (KernelStats * len(KERNEL_NAMES))()
        _check(self.lib.stn_profile_read(self.h, arr))
        return {name: {"launches": arr[i].launches, "ms": arr[i].ms, "bytes": arr[i].bytes,
                       "flops": arr[i].flops} for i, name in enumerate(KERNEL_NAMES)}

    def accum(self):
        h = C.c_void_p()
        _check(self.lib.stn_accum_create(self.h, C.byref(h)))
        return Accum(self, h)

    def reduce(self, batch, acc, stream=None):
        _check(self.lib.stn_reduce(self.h, batch.h, acc.h, stream if stream is not None else current_stream()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.stn_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def contract_many(plans, batches, stream=None):
    """Contracts batches of several whole-state-in-LDS plans in one launch
    (a device-side queue of (batch, trajectory) items)."""
    assert len(plans) == len(batches) and plans
    lib = plans[0].lib
    n = len(plans)
    ph = (C.c_void_p * n)(*[p.h for p in plans])
    bh = (C.c_void_p * n)(*[b.h for b in batches])
    _check(lib.stn_contract_many(ph, bh, n, stream if stream is not None else current_stream()))


class Batch:
    def __init__(self, plan, h, K):
        self.plan, self.h, self.K = plan, h, K

    def indices(self):
        out = np.zeros((self.K, self.plan.S), dtype=np.uint8)
        if self.plan.S:
            _check(self.plan.lib.stn_batch_indices(self.h, out.ctypes.data_as(C.POINTER(C.c_uint8))))
        return out

    def energies(self):
        e = np.zeros(self.K, dtype=np.float64)
        _check(self.plan.lib.stn_batch_results(self.h, e.ctypes.data_as(C.POINTER(C.c_double)), None))
        return e

    def states(self):
        st = np.zeros((self.K, 1 << self.plan.n), dtype=np.complex128)
        _check(self.plan.lib.stn_batch_results(self.h, None,
                                               st.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))))
        return st

    def close(self):
        if getattr(self, "h", None):
            self.plan.lib.stn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Accum:
    def __init__(self, plan, h):
        self.plan, self.h = plan, h

    def read(self, stream=None):
        r = Result()
        _check(self.plan.lib.stn_accum_read(self.h, C.byref(r), stream if stream is not None else current_stream()))
        N = 1 << self.plan.n
        out = {"k_done": r.k_done, "energy_mean": r.energy_mean, "energy_se": r.energy_se,
               "trace": r.trace_mean}
        if r.energies:
            out["energies"] = np.ctypeslib.as_array(r.energies, shape=(r.k_done,)).copy()
        if r.diag:
            out["diag"] = np.ctypeslib.as_array(r.diag, shape=(N,)).copy()
        if r.rho:
            out["rho"] = np.ctypeslib.as_array(r.rho, shape=(N * N * 2,)).copy().view(np.complex128).reshape(N, N)
        return out

    def sample(self, u, out=None, stream=None, no_alloc=False):
        """Bitstrings drawn from sigma_approx with the uniforms u (a float64
        device tensor); returns an int32 device tensor of basis indices.
        no_alloc=True calls stn_accum_sample_noalloc (the library allocates
        nothing; pass out to allocate nothing here either)."""
        import torch
        if not (u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
            raise ValueError("u must be a contiguous float64 device tensor")
        m = u.numel()
        if out is None:
            out = torch.empty(m, dtype=torch.int32, device=u.device)
        if out.numel() < m or out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 device tensor of at least u.numel() elements")
        fn = self.plan.lib.stn_accum_sample_noalloc if no_alloc else self.plan.lib.stn_accum_sample
        _check(fn(self.h, u.data_ptr(), m, out.data_ptr(), stream if stream is not None else current_stream()))
        return out[:m]

    def close(self):
        if getattr(self, "h", None):
            self.plan.lib.stn_accum_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate_batch_ensemble(problem, K=None, seed=None, outputs=OUT_ENERGY, precision=64, batch=None,
                            plan_kind=PLAN_AUTO, plan=None):
    """The ensemble of Sec. III-G for one job: plan, then sample / contract /
    reduce in batches of `batch` trajectories, then read the FP64 result."""
    K = K if K is not None else problem.K
    seed = seed if seed is not None else problem.seed
    pl = plan or Plan(problem, outputs=outputs, precision=precision, plan_kind=plan_kind)
    acc = pl.accum()
    step = batch or K
    for k0 in range(0, K, step):
        b = pl.sample(seed, k0, min(step, K - k0))
        pl.contract(b)
        pl.reduce(b, acc)
        b.close()
    res = acc.read()
    acc.close()
    return res


def _check_srv(st):
    if st != 0:
        raise StnError(st, _lib.stn_server_last_error().decode())


class Server:
    """stn_server_*: many <C> jobs of different circuits on one device, with
    continuous batching (jobs are admitted as device memory frees up and their
    chunks interleave).  Device memory comes from the server's own pool, not
    PyTorch's allocator; hbm_budget bounds it."""

    def __init__(self, hbm_budget=64 << 30, job_share=0.5, n_streams=3, max_active=16, plan_cache=64,
                 precision=64, chunk_max=0, drain_on_destroy=True, reserve_cus=32, graphs=False, gang=True):
        self.lib = load()
        o = ServerOpts()
        self.lib.stn_server_opts_default(C.byref(o))
        o.hbm_budget = int(hbm_budget)
        o.job_share = float(job_share)
        o.n_streams = n_streams
        o.max_active = max_active
        o.plan_cache = plan_cache
        o.precision = precision
        o.chunk_max = chunk_max
        o.drain_on_destroy = 1 if drain_on_destroy else 0
        o.reserve_cus = int(reserve_cus)
        o.graphs = 1 if graphs else 0
        o.gang = 1 if gang else 0
        h = C.c_void_p()
        _check_srv(self.lib.stn_server_create(C.byref(o), C.byref(h)))
        self.h = h

    def submit(self, problem, seed=None, K=None, tag=0):
        circ, noise, obs, keep = _problem_structs(problem, True)
        jid = C.c_uint64()
        _check_srv(self.lib.stn_server_submit(self.h, C.byref(circ), C.byref(noise), C.byref(obs),
                                              int(problem.seed if seed is None else seed),
                                              int(problem.K if K is None else K), int(tag), C.byref(jid)))
        return jid.value

    def poll(self, wait=0.0, cap=256):
        arr = (JobResult * cap)()
        n = C.c_uint32()
        _check_srv(self.lib.stn_server_poll(self.h, arr, cap, C.byref(n), float(wait)))
        out = []
        for i in range(n.value):
            r = arr[i]
            d = {f: getattr(r, f) for f, _ in JobResult._fields_ if f != "error"}
            d["error"] = r.error.decode(errors="replace")
            d["plan_name"] = PLAN_NAMES.get(d["plan_kind"], "?")
            out.append(d)
        return out

    def drain(self, timeout=3600.0):
        _check_srv(self.lib.stn_server_drain(self.h, float(timeout)))

    def stats(self):
        s = ServerStats()
        _check_srv(self.lib.stn_server_stats_read(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def clock(self):
        return self.lib.stn_server_clock(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.stn_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
