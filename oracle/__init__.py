"""QHap CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of the phasing hot path, written from the
paper's Methods section (equations numbered in order of appearance: (1)
ternary encoding, (2)-(3) read conflicts, (4)-(6) Ising / Max-Cut, (7)-(8)
vote counts, (9)-(14) SNP log-likelihood weights, (15)-(17) refinement and
parity).  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library and never
imports it.

Parity status per function (pins live in ``tests/test_oracle_*.py``):

* encode, read_graph, snp_graph, components, cuts/energy, select, greedy,
  phase_vote, phase_parity, flip_crossing, metrics, quantizers, init RNG,
  one bSB step: pinned (closed forms, hand tables, brute force, published
  test vectors, invariants).
* The final spins of a long bSB run are a heuristic's output: parity unpinned
  beyond the cut-gap / switch-error contract (brute-force optimum on <= 20
  nodes and the frustration-free planted optimum pin the cut itself).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "qh_oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, dbl, u64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    sig = {
        "or_num_threads": (i32, []),
        "or_encode": (None, [i64, P, P, P, P]),
        "or_read_graph_dense": (i32, [i32, i64, i64, P, P, P, P, P]),
        "or_snp_graph_structure": (i32, [i64, i64, P, P, P, i32, P, P]),
        "or_snp_graph_values": (i32, [i64, i64, P, P, P, P, P, i32, P, P, P]),
        "or_components": (i64, [i64, P, P, P]),
        "or_c0": (dbl, [i64, P, P]),
        "or_splitmix64": (u64, [u64, u64]),
        "or_init": (None, [u64, i64, i32, P, P]),
        "or_bsb_run": (None, [i64, P, P, P, i32, i64, i64, P, dbl, dbl, dbl, P, P]),
        "or_sb_run": (None, [i64, P, P, P, i32, i64, i64, P, dbl, dbl, dbl, P, P, i32, P]),
        "or_pump_linear": (None, [i64, P]),
        "or_signs": (None, [i64, P, P]),
        "or_cuts": (None, [i64, P, P, P, P, i64, i32, P, P]),
        "or_energy": (None, [i64, P, P, P, i32, P, P]),
        "or_select": (None, [i64, P, i64, i32, P, P, P, P]),
        "or_greedy": (i64, [i64, P, P, P, dbl, i64, P]),
        "or_phase_vote": (None, [i64, i64, P, P, P, P, P, P, P, P]),
        "or_phase_parity": (None, [i64, P, i64, P, P, P, P]),
        "or_flip_crossing": (None, [i64, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(_load().or_num_threads())


class CSR:
    """Structural-pair graph in CSR form (FP64 values, columns ascending)."""

    def __init__(self, n: int, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray):
        self.n = int(n)
        self.row_ptr = _c(row_ptr, np.int64)
        self.col = _c(col, np.int32)
        self.val = _c(val, np.float64)

    @property
    def nnz_struct(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def nnz(self) -> int:
        return int(np.count_nonzero(self.val))

    def dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d


# --------------------------------------------------------------------------
# Eq. (1)
# --------------------------------------------------------------------------

def encode(snp: np.ndarray, allele: np.ndarray, init_h1: np.ndarray) -> np.ndarray:
    snp = _c(snp, np.int32); allele = _c(allele, np.uint8); init_h1 = _c(init_h1, np.uint8)
    if snp.size and (int(snp.min()) < 0 or int(snp.max()) >= init_h1.shape[0]):
        raise ValueError("SNP index out of range")
    M = np.empty(snp.shape[0], dtype=np.int8)
    _load().or_encode(snp.shape[0], _p(snp), _p(allele), _p(init_h1), _p(M))
    return M


# --------------------------------------------------------------------------
# Eqs. (2)-(3): read graph
# --------------------------------------------------------------------------

def read_graph_dense(n_snp: int, frag_ptr, snp, M, kind: str = "signed") -> Tuple[np.ndarray, np.ndarray]:
    """Dense (weights int64, co-coverage int32) of the read graph."""
    frag_ptr = _c(frag_ptr, np.int64); snp = _c(snp, np.int32); M = _c(M, np.int8)
    nf = frag_ptr.shape[0] - 1
    W = np.empty((nf, nf), dtype=np.int64)
    C = np.empty((nf, nf), dtype=np.int32)
    k = {"conflict": 0, "signed": 1}[kind]
    rc = _load().or_read_graph_dense(k, n_snp, nf, _p(frag_ptr), _p(snp), _p(M), _p(W), _p(C))
    if rc:
        raise MemoryError("oracle read graph failed")
    return W, C


def read_graph(n_snp: int, frag_ptr, snp, M, kind: str = "signed") -> CSR:
    """Ising couplings J of the read graph over co-covered pairs.

    conflict: J = -A with A_ab the conflict count (Eq. 3, Eq. 4).
    signed:   J_ab = sum_j M_aj M_bj (agree minus disagree).
    """
    W, C = read_graph_dense(n_snp, frag_ptr, snp, M, kind)
    nf = W.shape[0]
    mask = C > 0
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(nf + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    np.cumsum(row_ptr, out=row_ptr)
    vals = W[rows, cols].astype(np.float64)
    if kind == "conflict":
        vals = -vals
    return CSR(nf, row_ptr, cols.astype(np.int32), vals)


# --------------------------------------------------------------------------
# Eqs. (9)-(14): SNP graph
# --------------------------------------------------------------------------

def snp_weights(n_snp: int, frag_ptr, snp, M, phred, alpha=None, linkage_k: int = 10) -> CSR:
    """Max-Cut edge weights w_uv of Eq. (14) over the linked SNP pairs."""
    frag_ptr = _c(frag_ptr, np.int64); snp = _c(snp, np.int32); M = _c(M, np.int8)
    phred = _c(phred, np.uint8)
    alpha = None if alpha is None else _c(alpha, np.float64)
    nf = frag_ptr.shape[0] - 1
    lib = _load()
    row_ptr = np.zeros(n_snp + 1, dtype=np.int64)
    rc = lib.or_snp_graph_structure(n_snp, nf, _p(frag_ptr), _p(snp), _p(phred), linkage_k,
                                    _p(row_ptr), None)
    if rc:
        raise MemoryError("oracle SNP structure failed")
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    rc = lib.or_snp_graph_structure(n_snp, nf, _p(frag_ptr), _p(snp), _p(phred), linkage_k,
                                    _p(row_ptr), _p(col))
    if rc:
        raise MemoryError("oracle SNP structure failed")
    val = np.empty(col.shape[0], dtype=np.float64)
    rc = lib.or_snp_graph_values(n_snp, nf, _p(frag_ptr), _p(snp), _p(M), _p(phred), _p(alpha),
                                 linkage_k, _p(row_ptr), _p(col), _p(val))
    if rc:
        raise MemoryError("oracle SNP values failed")
    return CSR(n_snp, row_ptr, col, val)


def snp_graph(n_snp: int, frag_ptr, snp, M, phred, alpha=None, linkage_k: int = 10) -> CSR:
    """Ising couplings J = -w of the SNP graph (Eq. 4 with A = w of Eq. 14)."""
    w = snp_weights(n_snp, frag_ptr, snp, M, phred, alpha, linkage_k)
    return CSR(n_snp, w.row_ptr, w.col, -w.val)


def build_graph(w, kind: str, linkage_k: int = 10) -> CSR:
    """Graph of a synthetic workload: kind in {read_signed, read_conflict, snp_llr}."""
    M = encode(w.snp, w.allele, w.init_h1)
    if kind == "read_signed":
        return read_graph(w.n_snp, w.frag_ptr, w.snp, M, "signed")
    if kind == "read_conflict":
        return read_graph(w.n_snp, w.frag_ptr, w.snp, M, "conflict")
    if kind == "snp_llr":
        return snp_graph(w.n_snp, w.frag_ptr, w.snp, M, w.phred, w.alpha, linkage_k)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# components, c0, init
# --------------------------------------------------------------------------

def components(g: CSR) -> Tuple[np.ndarray, int]:
    comp = np.empty(g.n, dtype=np.int32)
    nc = _load().or_components(g.n, _p(g.row_ptr), _p(g.col), _p(comp))
    return comp, int(nc)


def c0(g: CSR) -> float:
    return float(_load().or_c0(g.n, _p(g.row_ptr), _p(g.val)))


def splitmix64(seed: int, k: int) -> int:
    return int(_load().or_splitmix64(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.c_uint64(k)))


def init_state(seed: int, n: int, R: int) -> Tuple[np.ndarray, np.ndarray]:
    x = np.empty((n, R), dtype=np.float64)
    y = np.empty((n, R), dtype=np.float64)
    _load().or_init(ctypes.c_uint64(seed & (2**64 - 1)), n, R, _p(x), _p(y))
    return x, y


def pump_linear(steps: int) -> np.ndarray:
    p = np.empty(max(steps, 1), dtype=np.float64)
    _load().or_pump_linear(steps, _p(p))
    return p[:steps]


# --------------------------------------------------------------------------
# bSB
# --------------------------------------------------------------------------

def bsb_run(g: CSR, x: np.ndarray, y: np.ndarray, pump: np.ndarray, dt: float, c0_: float,
            a0: float = 1.0, k_begin: int = 0, k_end: Optional[int] = None, discrete: bool = False,
            field: Optional[np.ndarray] = None):
    """Advance (x, y) in place over steps [k_begin, k_end) of the pump table.

    ``discrete`` selects the discrete variant (dSB): the coupling uses sgn(x_j).  ``field``
    (length n) is the deformation term h: the coupling becomes c0 (J x + h)."""
    assert x.dtype == np.float64 and y.dtype == np.float64
    assert x.flags.c_contiguous and y.flags.c_contiguous
    n, R = x.shape
    pump = _c(pump, np.float64)
    if k_end is None:
        k_end = pump.shape[0]
    h = None if field is None else _c(field, np.float64)
    assert h is None or h.shape == (n,)
    _load().or_sb_run(g.n, _p(g.row_ptr), _p(g.col), _p(g.val), R, k_begin, k_end, _p(pump),
                      dt, c0_, a0, _p(x), _p(y), int(discrete), None if h is None else _p(h))
    return x, y


def bsb_step_dense(J: np.ndarray, x: np.ndarray, y: np.ndarray, p: float, dt: float, c0_: float,
                   a0: float = 1.0, walls: bool = True, discrete: bool = False,
                   field: Optional[np.ndarray] = None):
    """One bSB step in FP64 with a dense J, returning (x', y')."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xq = np.where(x >= 0.0, 1.0, -1.0) if discrete else x      # dSB: sgn(x), sgn(0) = +1
    z = np.asarray(J, dtype=np.float64) @ xq
    if field is not None:
        z = z + np.asarray(field, dtype=np.float64)[:, None]
    y2 = y + (-(a0 - p) * x + c0_ * z) * dt
    x2 = x + a0 * y2 * dt
    if not walls:
        return x2, y2
    wall = np.abs(x2) > 1.0
    x2 = np.where(wall, np.where(x2 > 0, 1.0, -1.0), x2)
    y2 = np.where(wall, 0.0, y2)
    return x2, y2


def signs(x: np.ndarray) -> np.ndarray:
    x = _c(x, np.float64)
    s = np.empty(x.shape, dtype=np.int8)
    _load().or_signs(x.size, _p(x), _p(s))
    return s


def cuts(g: CSR, comp: np.ndarray, n_comp: int, s: np.ndarray) -> np.ndarray:
    """cut[r, c] for spins s[n, R]."""
    s = _c(s, np.int8)
    if s.ndim == 1:
        s = s[:, None].copy()
    R = s.shape[1]
    comp = _c(comp, np.int32)
    out = np.empty((R, max(n_comp, 0)), dtype=np.float64)
    _load().or_cuts(g.n, _p(g.row_ptr), _p(g.col), _p(g.val), _p(comp), n_comp, R, _p(s), _p(out))
    return out


def energy(g: CSR, s: np.ndarray) -> np.ndarray:
    s = _c(s, np.int8)
    if s.ndim == 1:
        s = s[:, None].copy()
    R = s.shape[1]
    E = np.empty(R, dtype=np.float64)
    _load().or_energy(g.n, _p(g.row_ptr), _p(g.col), _p(g.val), R, _p(s), _p(E))
    return E


def select(comp: np.ndarray, n_comp: int, s: np.ndarray, cut: np.ndarray):
    s = _c(s, np.int8); comp = _c(comp, np.int32); cut = _c(cut, np.float64)
    n, R = s.shape
    best = np.empty(n, dtype=np.int8)
    best_r = np.empty(max(n_comp, 1), dtype=np.int32)
    _load().or_select(n, _p(comp), n_comp, R, _p(s), _p(cut), _p(best), _p(best_r))
    return best, best_r[:n_comp]


def greedy_eps(g: CSR, integer: bool) -> float:
    if integer:
        return 0.0
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    rs = np.zeros(g.n)
    np.add.at(rs, rows, np.abs(g.val))
    return 1e-12 * float(rs.max()) if g.n else 0.0


def greedy(g: CSR, s: np.ndarray, eps: float = 0.0, max_rounds: int = 100000):
    s = _c(s, np.int8).copy()
    rounds = _load().or_greedy(g.n, _p(g.row_ptr), _p(g.col), _p(g.val), eps, max_rounds, _p(s))
    return s, int(rounds)


# --------------------------------------------------------------------------
# phasing
# --------------------------------------------------------------------------

def phase_vote(n_snp: int, frag_ptr, snp, M, s_frag, comp_frag, init_h1):
    frag_ptr = _c(frag_ptr, np.int64); snp = _c(snp, np.int32); M = _c(M, np.int8)
    s_frag = _c(s_frag, np.int8); comp_frag = _c(comp_frag, np.int32); init_h1 = _c(init_h1, np.uint8)
    h1 = np.empty(n_snp, dtype=np.int8)
    block = np.empty(n_snp, dtype=np.int32)
    _load().or_phase_vote(n_snp, frag_ptr.shape[0] - 1, _p(frag_ptr), _p(snp), _p(M), _p(s_frag),
                          _p(comp_frag), _p(init_h1), _p(h1), _p(block))
    return h1, block


def phase_parity(comp, n_comp: int, s, init_h1):
    comp = _c(comp, np.int32); s = _c(s, np.int8); init_h1 = _c(init_h1, np.uint8)
    n = comp.shape[0]
    h1 = np.empty(n, dtype=np.int8)
    block = np.empty(n, dtype=np.int32)
    _load().or_phase_parity(n, _p(comp), n_comp, _p(s), _p(init_h1), _p(h1), _p(block))
    return h1, block


def flip_crossing(g: CSR, s) -> CSR:
    s = _c(s, np.int8)
    val = g.val.copy()
    _load().or_flip_crossing(g.n, _p(g.row_ptr), _p(g.col), _p(val), _p(s))
    return CSR(g.n, g.row_ptr, g.col, val)


def deformation_field(seed: int, n: int, R: int, attempt: int, amplitude: float) -> np.ndarray:
    """Deformation term h of refinement attempt ``attempt`` (1, 2, ...): the adaptive
    strategy of the SNP-based method (Methods) perturbs a stuck round with a field.  The
    paper gives no formula; this reading draws h_i = amplitude (2 u_i - 1) with u_i the
    SplitMix64 output of the round's seed at draw 2 n R + (attempt - 1) n + i (the draws
    after those of the initial state) mapped to [0, 1) by its top 53 bits."""
    k0 = 2 * n * R + (attempt - 1) * n
    u = np.array([(splitmix64(seed, k0 + i) >> 11) * 2.0 ** -53 for i in range(n)], dtype=np.float64)
    return amplitude * (2.0 * u - 1.0)


def refine(g: CSR, init_h1: np.ndarray, R: int, steps: int, dt: float = 0.5, seed: int = 0,
           max_rounds: int = 15, integer: bool = False, greedy_pass: bool = True,
           deform: float = 0.0, deform_tries: int = 0) -> Dict[str, object]:
    """Iterative refinement of the SNP-based method (Eqs. 15-17).

    Round t solves the current graph (seed + t).  With deform > 0, while a component still
    being refined has a negative cut, the round is solved again (at most deform_tries
    times, same seed) under the deformation field of amplitude deform / c0 (so that the
    force c0 h_i stays within deform), and each such component takes the new spins when
    their cut is higher (the adaptive strategy of the Methods for persistent negative
    cuts).  A component stops when its cut is not positive or its partition puts every
    vertex on one side; otherwise the vertices of its smaller subset (the s = -1 subset on
    a tie) add one to their flip counter C and every edge crossing the partition changes
    sign.  Haplotype 1 is H1 where C is even and H2 where C is odd.
    """
    comp, nc = components(g)
    C = np.zeros(g.n, dtype=np.int64)
    done = np.zeros(nc, dtype=bool)
    cur = g
    round_cuts = []
    rounds = 0
    deformed = 0
    for t in range(max_rounds):
        if done.all():
            break
        r = solve(cur, R, steps, dt, seed=seed + t, integer=integer, greedy_pass=greedy_pass)
        s = r["best"].copy()
        cut_c = cuts(cur, comp, nc, s)[0] if nc else np.zeros(0)
        for a in range(1, deform_tries + 1 if deform > 0 else 1):
            stuck = [c for c in range(nc) if not done[c] and cut_c[c] < 0]
            if not stuck:
                break
            h = deformation_field(seed + t, g.n, R, a, deform / r["c0"])
            r2 = solve(cur, R, steps, dt, seed=seed + t, integer=integer, greedy_pass=greedy_pass, field=h)
            deformed += 1
            cut2 = cuts(cur, comp, nc, r2["best"])[0]
            for c in stuck:
                if cut2[c] > cut_c[c]:
                    s[comp == c] = r2["best"][comp == c]
                    cut_c[c] = cut2[c]
        s_eff = np.ones(g.n, dtype=np.int8)
        applied = 0.0
        for c in range(nc):
            if done[c]:
                continue
            members = comp == c
            sc = s[members]
            if cut_c[c] <= 0 or np.all(sc == sc[0]):
                done[c] = True
                continue
            plus = int(np.count_nonzero(sc > 0))
            smin = 1 if plus < sc.shape[0] - plus else -1
            C[members & (s == smin)] += 1
            s_eff[members] = s[members]
            applied += cut_c[c]
        if not (s_eff < 0).any():
            break
        cur = flip_crossing(cur, s_eff)
        round_cuts.append(applied)
        rounds += 1
    h1 = np.where(comp >= 0, np.where(C % 2 == 1, 1 - init_h1.astype(np.int64), init_h1), -1).astype(np.int8)
    block = np.where(comp >= 0, comp, -1).astype(np.int32)
    return dict(h1=h1, block=block, flips=C, rounds=rounds, round_cuts=round_cuts, comp=comp,
                n_comp=nc, deformed=deformed)


# --------------------------------------------------------------------------
# whole solve, as the library's bsb_solve defines it
# --------------------------------------------------------------------------

def merge_best(g: CSR, comp: np.ndarray, n_comp: int, spin_sets):
    """Best sample seen so far per component (the best-of-many-samples rule of the SB
    solution, applied over several readouts of one run): over a sequence of spin sets
    s_e [n, R], component c keeps the (e, r) with the largest cut, ties going to the
    earlier readout, then the lower replica; returns (spins oriented so that the
    component's lowest vertex reads +1, cut per component, replica per component)."""
    best = np.ones(g.n, dtype=np.int8)
    best_cut = np.full(max(n_comp, 0), -np.inf)
    best_rep = np.zeros(max(n_comp, 0), dtype=np.int32)
    for s in spin_sets:
        cut = cuts(g, comp, n_comp, s)                       # [R, n_comp]
        pick, pick_r = select(comp, n_comp, s, cut)
        for c in range(n_comp):
            v = cut[pick_r[c], c]
            if v > best_cut[c]:
                best_cut[c] = v
                best_rep[c] = pick_r[c]
                best[comp == c] = pick[comp == c]
    return best, best_cut, best_rep


def solve(g: CSR, R: int, steps: int, dt: float = 0.5, c0_: Optional[float] = None,
          a0: float = 1.0, seed: int = 0, greedy_pass: bool = True, integer: bool = False,
          x0: Optional[np.ndarray] = None, y0: Optional[np.ndarray] = None,
          pump: Optional[np.ndarray] = None, discrete: bool = False,
          field: Optional[np.ndarray] = None, eval_every: int = 0) -> Dict[str, object]:
    """Whole solve: bSB steps, signs, FP64 cuts, best replica per component, greedy pass.

    ``eval_every`` = m > 0 reads the signs out after every m steps (and after the last):
    each component keeps its best sample over all readouts (``merge_best``), and the Ising
    energy -1/2 s'Js (Eq. 5) of every replica at every readout is returned as ``energy``
    [n_eval, R].  With m = 0 there is one readout, after the last step."""
    comp, nc = components(g)
    if c0_ is None or c0_ <= 0:
        c0_ = c0(g)
    if x0 is None:
        x, y = init_state(seed, g.n, R)
    else:
        x = np.array(x0, dtype=np.float64, order="C")
        y = np.array(y0, dtype=np.float64, order="C")
    if pump is None:
        pump = pump_linear(steps)
    marks = list(range(eval_every, steps, eval_every)) if eval_every > 0 else []
    marks.append(steps)
    spin_sets, energy_rows = [], []
    k = 0
    for k1 in marks:
        bsb_run(g, x, y, pump, dt, c0_, a0, k, k1, discrete=discrete, field=field)
        k = k1
        spin_sets.append(signs(x))
        energy_rows.append(energy(g, spin_sets[-1]))
    s = spin_sets[-1]
    cut = cuts(g, comp, nc, s)
    best, best_c, best_r = merge_best(g, comp, nc, spin_sets)
    sel_cut = float(sum(best_c[c] for c in range(nc)))
    rounds = 0
    if greedy_pass:
        best, rounds = greedy(g, best, greedy_eps(g, integer))
    final = float(cuts(g, comp, nc, best).sum())
    return dict(comp=comp, n_comp=nc, c0=c0_, x=x, y=y, spins=s, cuts=cut.sum(axis=1),
                cut_rc=cut, best=best, best_r=best_r, selected_cut=sel_cut, best_cut=final,
                greedy_rounds=rounds, energy=np.array(energy_rows), eval_steps=marks)
