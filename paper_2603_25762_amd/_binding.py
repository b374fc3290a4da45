"""ctypes marshalling for ``include/qhap.h``."""
from __future__ import annotations

import ctypes
import enum
import json
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "lib", "libqhap.so")

KIND = {"read_conflict": 0, "read_signed": 1, "snp_llr": 2}
STORAGE = {"dense": 0, "skyline": 1}
DTYPE = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}


class Status(enum.IntEnum):
    OK = 0
    EINVAL = 1
    ENOMEM = 2
    EHIP = 3
    EUNSUPPORTED = 4
    ENUMERIC = 5


class QhapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{Status(status).name}: {message}")
        self.status = Status(status)


P = ctypes.c_void_p


class _Reads(ctypes.Structure):
    _fields_ = [("n_frag", ctypes.c_int64), ("frag_ptr", P), ("snp", P), ("allele", P),
                ("phred", P), ("alpha", P)]


class _Snps(ctypes.Structure):
    _fields_ = [("n_snp", ctypes.c_int32), ("init_h1", P)]


class _GraphOpts(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("storage", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("linkage_k", ctypes.c_int32), ("band_limit", ctypes.c_int32),
                ("max_device_bytes", ctypes.c_int64), ("deterministic", ctypes.c_int32)]


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_snp", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_comp", ctypes.c_int64),
                ("stored_entries", ctypes.c_int64), ("stored_bytes", ctypes.c_int64),
                ("longrange_nnz", ctypes.c_int64), ("dense_tiles", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("kind", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("integer_weights", ctypes.c_int32), ("c0_auto", ctypes.c_double),
                ("band_dtype", ctypes.c_int32), ("total_weight", ctypes.c_double),
                ("largest_component", ctypes.c_int64)]


class _BsbOpts(ctypes.Structure):
    _fields_ = [("replicas", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("step_begin", ctypes.c_int32), ("step_end", ctypes.c_int32),
                ("dt", ctypes.c_double), ("c0", ctypes.c_double), ("a0", ctypes.c_double),
                ("pump", P), ("seed", ctypes.c_uint64), ("init", ctypes.c_int32),
                ("readout", ctypes.c_int32), ("greedy", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("plan", ctypes.c_int32),
                ("replica_tile", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("tiles_in_flight", ctypes.c_int32), ("persistent_sync", ctypes.c_int32),
                ("field", P), ("eval_every", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("best_spins", P), ("cuts", P), ("cut_rc", P),
                ("best_replica", P), ("selected_cut", P), ("best_cut", P), ("all_spins", P),
                ("greedy_rounds", P), ("best_energy", P), ("energy", P)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("plan_used", ctypes.c_int32), ("persistent_ok", ctypes.c_int32),
                ("replicas_per_group", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("workgroups_per_group", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("us_per_step", ctypes.c_float * 2), ("replica_tile", ctypes.c_int32),
                ("tiles_in_flight", ctypes.c_int32), ("skyline_kernel", ctypes.c_int32),
                ("skyline_us", ctypes.c_float * 2), ("persistent_sync", ctypes.c_int32),
                ("us_persistent_coherent", ctypes.c_float)]


class _Schedule(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("samples", ctypes.c_int32), ("replicas", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("size", ctypes.c_int64)]


class _BatchedResult(ctypes.Structure):
    _fields_ = [("best_spins", P), ("cuts", P), ("best_cut", P), ("selected_cut", P),
                ("x", P), ("y", P), ("plan_used", ctypes.c_int32)]


_lib = None


def load():
    """Load the built library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise ImportError(f"HIP library not built: {lib_path} is missing "
                          "(run __graft_entry__.build())")
    lib = ctypes.CDLL(lib_path)
    I = ctypes.c_int
    sig = {
        "qh_build_graph": [ctypes.POINTER(_Reads), ctypes.POINTER(_Snps), ctypes.POINTER(_GraphOpts),
                           ctypes.POINTER(P), P],
        "qh_build_graphs": [ctypes.c_int64, ctypes.POINTER(_Reads), ctypes.POINTER(_Snps),
                            ctypes.POINTER(_GraphOpts), ctypes.POINTER(P), ctypes.c_int32, P],
        "qh_graph_free": [P],
        "qh_graph_get_info": [P, ctypes.POINTER(_GraphInfo)],
        "qh_graph_export_rows": [P, ctypes.c_int64, ctypes.c_int64, P, P],
        "qh_graph_export_stored_rows": [P, ctypes.c_int64, ctypes.c_int64, P, P],
        "qh_graph_components": [P, P, P],
        "qh_bsb_solve": [P, ctypes.POINTER(_BsbOpts), ctypes.POINTER(_Result), P],
        "qh_bsb_solve_batched": [P, ctypes.c_int32, ctypes.POINTER(_BsbOpts),
                                 ctypes.POINTER(_BatchedResult), P],
        "qh_phase": [P, P, P, P, P],
        "qh_phase_noalloc": [P, P, P, P, P],
        "qh_phase_batched": [P, ctypes.c_int32, P, P, P, P],
        "qh_flip_crossing": [P, P, P],
        "qh_refine": [P, ctypes.POINTER(_BsbOpts), ctypes.c_int32, ctypes.c_float, ctypes.c_int32, P, P, P,
                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                      ctypes.POINTER(ctypes.c_int32), P],
        "qh_solve_plan_info": [P, ctypes.c_int32, ctypes.POINTER(_PlanInfo)],
        "qh_autotune": [P, ctypes.POINTER(_BsbOpts), ctypes.POINTER(_BsbOpts), ctypes.POINTER(ctypes.c_float),
                        ctypes.c_char_p, P],
        "qh_adaptive_schedule": [ctypes.c_int64, ctypes.POINTER(_Schedule)],
        "qh_release_cached_memory": [ctypes.POINTER(ctypes.c_int64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = I
    lib.qh_last_error.restype = ctypes.c_char_p
    lib.qh_last_error.argtypes = []
    lib.qh_version.restype = ctypes.c_char_p
    lib.qh_version.argtypes = []
    _lib = lib
    return lib


def version() -> str:
    return load().qh_version().decode()


def release_cached_memory() -> int:
    """Hands the library's cached idle device blocks back to the device; returns the bytes."""
    out = ctypes.c_int64(0)
    _check(load().qh_release_cached_memory(ctypes.byref(out)))
    return out.value


def _check(rc: int):
    if rc != 0:
        raise QhapError(rc, load().qh_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


class Graph:
    """Owns a ``qh_graph*``; freed when garbage-collected or by :meth:`free`."""

    def __init__(self, handle: int, keep=()):
        self._h = ctypes.c_void_p(handle)
        self._keep = keep
        self._n_snp = None

    @property
    def n_snp(self) -> int:
        """SNP count of the graph's inputs (fixed for the graph's life; read once)."""
        if self._n_snp is None:
            self._n_snp = int(self.info()["n_snp"])
        return self._n_snp

    @property
    def handle(self):
        return self._h

    def info(self) -> Dict[str, object]:
        inf = _GraphInfo()
        _check(load().qh_graph_get_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in _GraphInfo._fields_}

    def export_rows(self, row0: int, row1: int, stored: bool = False) -> torch.Tensor:
        n = self.info()["n"]
        out = torch.empty((row1 - row0, n), dtype=torch.float64, device="cuda")
        fn = load().qh_graph_export_stored_rows if stored else load().qh_graph_export_rows
        _check(fn(self._h, row0, row1, _ptr(out), _stream()))
        return out

    def components(self) -> torch.Tensor:
        n = self.info()["n"]
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(load().qh_graph_components(self._h, _ptr(out), _stream()))
        return out

    def plan_info(self, replicas: int) -> Dict[str, object]:
        """Step-loop plan of earlier solves with this replica count (autotuner report)."""
        pi = _PlanInfo()
        _check(load().qh_solve_plan_info(self._h, replicas, ctypes.byref(pi)))
        d = {name: getattr(pi, name) for name, _ in _PlanInfo._fields_}
        d["us_per_step"] = list(pi.us_per_step)
        d["skyline_us"] = list(pi.skyline_us)
        return d

    def free(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            _check(load().qh_graph_free(self._h))
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        # No HIP call while the interpreter shuts down: by then a profiler or the runtime may
        # already have torn down (the process releases device memory on exit anyway).
        try:
            import sys
            if sys.is_finalizing():
                return
            if self._h is not None and self._h.value and _lib is not None:
                _lib.qh_graph_free(self._h)
                self._h = ctypes.c_void_p(0)
        except Exception:
            pass


def _build_args(frag_ptr: torch.Tensor, snp: torch.Tensor, allele: torch.Tensor,
                phred: Optional[torch.Tensor], init_h1: torch.Tensor, *, kind: str = "read_signed",
                storage: Optional[str] = None, dtype: str = "f32",
                alpha: Optional[torch.Tensor] = None, linkage_k: int = 10,
                band_limit: int = 0, max_device_bytes: int = 0, deterministic: bool = False):
    if storage is None:
        storage = "skyline" if kind == "snp_llr" else "dense"
    for t, dt in ((frag_ptr, torch.int64), (snp, torch.int32), (allele, torch.uint8),
                  (init_h1, torch.uint8)):
        if t.dtype != dt:
            raise TypeError(f"expected {dt}, got {t.dtype}")
    if phred is not None and phred.dtype != torch.uint8:
        raise TypeError("phred must be uint8")
    if alpha is not None and alpha.dtype != torch.float64:
        raise TypeError("alpha must be float64")
    reads = _Reads(frag_ptr.numel() - 1, _ptr(frag_ptr), _ptr(snp), _ptr(allele), _ptr(phred),
                   _ptr(alpha))
    snps = _Snps(init_h1.numel(), _ptr(init_h1))
    opts = _GraphOpts(KIND[kind], STORAGE[storage], DTYPE[dtype], linkage_k, band_limit, max_device_bytes,
                      int(deterministic))
    return reads, snps, opts


def build_graph(frag_ptr: torch.Tensor, snp: torch.Tensor, allele: torch.Tensor,
                phred: Optional[torch.Tensor], init_h1: torch.Tensor, *, kind: str = "read_signed",
                storage: Optional[str] = None, dtype: str = "f32",
                alpha: Optional[torch.Tensor] = None, linkage_k: int = 10,
                band_limit: int = 0, max_device_bytes: int = 0, deterministic: bool = False,
                stream=None) -> Graph:
    reads, snps, opts = _build_args(frag_ptr, snp, allele, phred, init_h1, kind=kind, storage=storage,
                                    dtype=dtype, alpha=alpha, linkage_k=linkage_k, band_limit=band_limit,
                                    max_device_bytes=max_device_bytes, deterministic=deterministic)
    h = ctypes.c_void_p()
    _check(load().qh_build_graph(ctypes.byref(reads), ctypes.byref(snps), ctypes.byref(opts),
                                 ctypes.byref(h), _stream(stream)))
    return Graph(h.value)


def build_graphs(specs: Sequence[Dict[str, object]], *, threads: int = 0, stream=None) -> List[Graph]:
    """Many graphs in one call (qh_build_graphs, host threads each on a stream of its own).
    ``specs``: one dict of build_graph's arguments per graph (frag_ptr, snp, allele, phred,
    init_h1 and any of its keyword arguments but stream)."""
    n = len(specs)
    if n == 0:
        return []
    reads = (_Reads * n)()
    snps = (_Snps * n)()
    opts = (_GraphOpts * n)()
    for i, sp in enumerate(specs):
        reads[i], snps[i], opts[i] = _build_args(**sp)
    out = (ctypes.c_void_p * n)()
    _check(load().qh_build_graphs(n, reads, snps, opts, out, threads, _stream(stream)))
    return [Graph(out[i]) for i in range(n)]


def _check_field(field: Optional[torch.Tensor], n: int):
    if field is None:
        return
    if field.dtype != torch.float32 or field.device.type != "cuda" or not field.is_contiguous():
        raise TypeError("field must be a contiguous float32 device tensor")
    if field.numel() != n:
        raise ValueError(f"field holds {field.numel()} values for {n} vertices")


def adaptive_schedule(size) -> Dict[str, int]:
    """The library's size-adaptive bSB settings (qh_adaptive_schedule): steps, samples,
    replicas, max_rounds and the size the rule was applied to.  ``size`` is a vertex count,
    or a Graph, whose largest component is used."""
    if isinstance(size, Graph):
        size = size.info()["largest_component"]
    sc = _Schedule()
    _check(load().qh_adaptive_schedule(int(size), ctypes.byref(sc)))
    return {name: int(getattr(sc, name)) for name, _ in _Schedule._fields_}


def bsb_solve(g: Graph, replicas: int, steps: int, *, dt: float = 0.5, c0: float = 0.0,
              a0: float = 1.0, pump: Optional[torch.Tensor] = None, seed: int = 0,
              init: bool = True, x: Optional[torch.Tensor] = None, y: Optional[torch.Tensor] = None,
              step_begin: int = 0, step_end: int = 0, readout: bool = True, greedy: bool = True,
              use_graph: bool = False, all_spins: bool = False, per_component: bool = False,
              plan: int = 0, replica_tile: int = 0, discrete: bool = False, tiles_in_flight: int = 0,
              persistent_sync: int = 0, field: Optional[torch.Tensor] = None, eval_every: int = 0,
              energy: bool = False, out: Optional[Dict[str, torch.Tensor]] = None,
              stream=None) -> Dict[str, torch.Tensor]:
    """Runs bSB; returns device tensors (best_spins, cuts, best_cut, selected_cut, ...).

    ``x``/``y`` (float32 [n, R]) give the starting state when ``init`` is False and
    receive the final state when passed.  ``field`` (float32 [n], device) is the
    deformation term h added to every row's coupling sum.  ``eval_every`` > 0 reads the
    spins out every that many steps and keeps each component's best so far; ``energy``
    returns the Ising energy of every replica at each evaluation (float64 [n_eval, R]).
    ``out`` may supply preallocated result tensors (keys as returned) so that repeated
    calls allocate nothing.
    """
    inf = g.info()
    n, nc = inf["n"], inf["n_comp"]
    _check_field(field, n)
    dev = "cuda"
    res = {} if out is None else dict(out)
    keep = {}

    def alloc(key, shape, dtype, zero=False):
        # buffers never have zero elements, so the library never sees a NULL pointer
        if key in res:
            keep[key] = res[key]
            return
        full = (torch.zeros if zero else torch.empty)(tuple(max(s, 1) for s in shape), dtype=dtype,
                                                      device=dev)
        keep[key] = full
        res[key] = full[tuple(slice(0, s) for s in shape)]

    if readout:
        alloc("best_spins", (n,), torch.int8)
        alloc("cuts", (replicas,), torch.float64)
        alloc("best_cut", (1,), torch.float64)
        alloc("selected_cut", (1,), torch.float64)
        alloc("greedy_rounds", (1,), torch.int32, zero=True)
        alloc("best_energy", (1,), torch.float64)
        if all_spins:
            alloc("all_spins", (n, replicas), torch.int8)
        if per_component:
            alloc("cut_rc", (replicas, nc), torch.float64)
            alloc("best_replica", (nc,), torch.int32)
        if energy:
            span = (step_end or steps) - step_begin
            n_eval = max(1, -(-span // eval_every)) if eval_every > 0 else 1
            alloc("energy", (n_eval, replicas), torch.float64)
    if x is not None:
        res["x"] = x
    if y is not None:
        res["y"] = y
    if pump is not None:
        res["pump"] = pump
    opts = _BsbOpts(replicas, steps, step_begin, step_end, dt, c0, a0, _ptr(pump), seed & (2**64 - 1),
                    int(init), int(readout), int(greedy), int(use_graph), int(plan), int(replica_tile),
                    int(discrete), int(tiles_in_flight), int(persistent_sync), _ptr(field), int(eval_every))
    r = _Result(_ptr(x), _ptr(y), _ptr(keep.get("best_spins")), _ptr(keep.get("cuts")),
                _ptr(keep.get("cut_rc")), _ptr(keep.get("best_replica")), _ptr(keep.get("selected_cut")),
                _ptr(keep.get("best_cut")), _ptr(keep.get("all_spins")), _ptr(keep.get("greedy_rounds")),
                _ptr(keep.get("best_energy")), _ptr(keep.get("energy")))
    _check(load().qh_bsb_solve(g.handle, ctypes.byref(opts), ctypes.byref(r), _stream(stream)))
    return res


def energy_trace(g: Graph, replicas: int, steps: int, every: int, *, dt: float = 0.5, c0: float = 0.0,
                 a0: float = 1.0, seed: int = 0, discrete: bool = False, plan: int = 1,
                 stream=None) -> Dict[str, object]:
    """Ising energy (Eq. 5) of every replica's signs every `every` steps of one schedule
    (the convergence view of the solver comparison): one solve with eval_every = every,
    read out without the greedy pass.  Returns steps (the step count of each evaluation),
    energy (float64 [len(steps), replicas]) and best (the lowest energy per evaluation)."""
    if every < 1 or steps < 1:
        raise ValueError("steps and every must be >= 1")
    r = bsb_solve(g, replicas, steps, dt=dt, c0=c0, a0=a0, seed=seed, greedy=False, discrete=discrete,
                  plan=plan, eval_every=every, energy=True, stream=stream)
    energy = r["energy"].cpu().numpy()
    marks = [min(steps, (e + 1) * every) for e in range(energy.shape[0])]
    return dict(steps=marks, energy=energy, best=energy.min(axis=1))


_TUNED = ("plan", "replica_tile", "tiles_in_flight", "persistent_sync")


def autotune(g: Graph, replicas: int, steps: int, *, dt: float = 0.5, c0: float = 0.0, a0: float = 1.0,
             discrete: bool = False, cache_path: Optional[str] = None, stream=None) -> Dict[str, object]:
    """Runs the plan-0 autotuner for (graph, replicas) on its own and returns the chosen
    options (keys plan, replica_tile, tiles_in_flight, persistent_sync: pass them to
    bsb_solve to skip tuning) plus us_per_step; with cache_path, appends them as one JSON
    line for load_tuned."""
    opts = _BsbOpts(replicas, steps, 0, 0, dt, c0, a0, None, 0, 1, 0, 0, 0, 0, 0, int(discrete), 0, 0, None, 0)
    chosen = _BsbOpts()
    us = (ctypes.c_float * 2)()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(load().qh_autotune(g.handle, ctypes.byref(opts), ctypes.byref(chosen), us, path, _stream(stream)))
    out = {k: int(getattr(chosen, k)) for k in _TUNED}
    out["us_per_step"] = [float(us[0]), float(us[1])]
    return out


def load_tuned(cache_path: str, g: Graph, replicas: int) -> Optional[Dict[str, int]]:
    """The options of the last line of an autotune cache written for a graph of this shape
    (n, nnz, kind, storage, dtype, dense_tiles) and replica count, or None."""
    inf = g.info()
    found = None
    with open(cache_path) as f:
        for line in f:
            rec = json.loads(line)
            if rec["replicas"] == replicas and all(rec[k] == inf[k] for k in ("n", "nnz", "kind", "storage", "dtype",
                                                                              "dense_tiles")):
                found = {k: int(rec[k]) for k in _TUNED}
    return found


def bsb_solve_batched(graphs: Sequence[Graph], replicas: int, steps: int, *, dt: float = 0.5,
                      c0: float = 0.0, a0: float = 1.0, seed: int = 0, greedy: bool = True,
                      use_graph: bool = False, plan: int = 0, return_state: bool = False,
                      discrete: bool = False, field: Optional[torch.Tensor] = None, readout: bool = True,
                      stream=None) -> Dict[str, torch.Tensor]:
    """All graphs in one launch; per-block results packed at ``vertex_offset`` / ``b * replicas``.

    ``field`` (float32 [sum n], device) is packed the same way: block b's deformation
    term from ``vertex_offset[b]``.  ``readout`` False runs the dynamics only."""
    ns = [g.info()["n"] for g in graphs]
    total = int(sum(ns))
    _check_field(field, total)
    nb = len(graphs)
    dev = "cuda"
    res = dict(best_spins=torch.empty(max(total, 1), dtype=torch.int8, device=dev),
               cuts=torch.empty(max(nb * replicas, 1), dtype=torch.float64, device=dev),
               best_cut=torch.empty(max(nb, 1), dtype=torch.float64, device=dev),
               selected_cut=torch.empty(max(nb, 1), dtype=torch.float64, device=dev))
    if return_state:
        res["x"] = torch.empty(max(total * replicas, 1), dtype=torch.float32, device=dev)
        res["y"] = torch.empty(max(total * replicas, 1), dtype=torch.float32, device=dev)
    arr = (ctypes.c_void_p * max(nb, 1))(*[g.handle.value for g in graphs])
    opts = _BsbOpts(replicas, steps, 0, 0, dt, c0, a0, None, seed & (2**64 - 1), 1, int(readout), int(greedy),
                    int(use_graph), plan, 0, int(discrete), 0, 0, _ptr(field), 0)
    r = _BatchedResult(_ptr(res["best_spins"]), _ptr(res["cuts"]), _ptr(res["best_cut"]),
                       _ptr(res["selected_cut"]), _ptr(res.get("x")), _ptr(res.get("y")), 0)
    _check(load().qh_bsb_solve_batched(arr, nb, ctypes.byref(opts), ctypes.byref(r), _stream(stream)))
    res["vertex_offset"] = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    res["plan_used"] = r.plan_used
    return res


def phase(g: Graph, spins: torch.Tensor, n_snp: Optional[int] = None, stream=None, noalloc: bool = False,
          out=None):
    """Haplotype 1 allele per SNP (-1 = unphased) and the phase-block label per SNP.

    ``noalloc`` calls qh_phase_noalloc (no device allocation inside the library); ``out``
    may supply the (h1, block) tensors."""
    if spins.dtype != torch.int8:
        raise TypeError("spins must be int8")
    if n_snp is None:
        n_snp = g.n_snp
    elif n_snp != g.n_snp:
        raise ValueError(f"n_snp = {n_snp}, the graph has {g.n_snp} SNPs")
    if out is None:
        h1 = torch.empty(max(n_snp, 1), dtype=torch.int8, device="cuda")
        block = torch.empty(max(n_snp, 1), dtype=torch.int32, device="cuda")
    else:
        h1, block = out
        if h1.dtype != torch.int8 or block.dtype != torch.int32 or h1.numel() < n_snp or block.numel() < n_snp:
            raise ValueError(f"out must be int8 and int32 tensors of at least {n_snp} elements")
    fn = load().qh_phase_noalloc if noalloc else load().qh_phase
    _check(fn(g.handle, _ptr(spins), _ptr(h1), _ptr(block), _stream(stream)))
    return h1[:n_snp], block[:n_snp]


def phase_batched(graphs: Sequence[Graph], spins: torch.Tensor, stream=None):
    """qh_phase_batched: every graph of a batched solve phased in one call.  ``spins`` packed as
    bsb_solve_batched's best_spins; returns (h1, block, snp_offset): graph b's SNPs are
    h1[snp_offset[b]:snp_offset[b + 1]] (and the same of block)."""
    if spins.dtype != torch.int8:
        raise TypeError("spins must be int8")
    nb = len(graphs)
    ns = [g.n_snp for g in graphs]
    so = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    total = int(so[-1])
    h1 = torch.empty(max(total, 1), dtype=torch.int8, device="cuda")
    block = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
    if nb:
        arr = (ctypes.c_void_p * nb)(*[g.handle.value for g in graphs])
        _check(load().qh_phase_batched(arr, nb, _ptr(spins), _ptr(h1), _ptr(block), _stream(stream)))
    return h1[:total], block[:total], so


def refine_adaptive(g: Graph, *, seed: int = 0, deform: float = 0.0, deform_tries: int = 0,
                    stream=None) -> Dict[str, object]:
    """The SNP-based method with its size-adaptive settings (adaptive_schedule: steps by
    graph size, 128 replicas for the 100 samples, up to 15 rounds) and, with deform > 0,
    the deformation of rounds stuck at a negative cut.  Returns refine's outputs plus the
    settings used."""
    a = adaptive_schedule(g)
    out = refine(g, a["replicas"], a["steps"], max_rounds=a["max_rounds"], seed=seed, deform=deform,
                 deform_tries=deform_tries, stream=stream)
    out["schedule"] = a
    return out


def flip_crossing(g: Graph, spins: torch.Tensor, stream=None):
    _check(load().qh_flip_crossing(g.handle, _ptr(spins), _stream(stream)))


def refine(g: Graph, replicas: int, steps: int, *, max_rounds: int = 15, dt: float = 0.5, c0: float = 0.0,
           a0: float = 1.0, seed: int = 0, greedy: bool = True, use_graph: bool = False, plan: int = 0,
           discrete: bool = False, deform: float = 0.0, deform_tries: int = 0,
           stream=None) -> Dict[str, object]:
    """Multi-round SNP refinement: h1, block (device), flips (device), round_cuts, rounds,
    deformed (re-solves under the deformation field, taken while a component's cut is
    negative: at most ``deform_tries`` per round, field amplitude ``deform / c0``)."""
    inf = g.info()
    n, n_snp = inf["n"], inf["n_snp"]
    h1 = torch.empty(max(n_snp, 1), dtype=torch.int8, device="cuda")
    block = torch.empty(max(n_snp, 1), dtype=torch.int32, device="cuda")
    flips = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    rc = (ctypes.c_double * max_rounds)()
    rounds = ctypes.c_int32(0)
    deformed = ctypes.c_int32(0)
    opts = _BsbOpts(replicas, steps, 0, 0, dt, c0, a0, None, seed & (2**64 - 1), 1, 1, int(greedy),
                    int(use_graph), plan, 0, int(discrete), 0, 0, None, 0)
    _check(load().qh_refine(g.handle, ctypes.byref(opts), max_rounds, float(deform), int(deform_tries), _ptr(h1),
                            _ptr(block), _ptr(flips), rc, ctypes.byref(rounds), ctypes.byref(deformed),
                            _stream(stream)))
    k = rounds.value
    return dict(h1=h1[:n_snp], block=block[:n_snp], flips=flips[:n], round_cuts=list(rc[:k]), rounds=k,
                deformed=deformed.value)
