"""Seeded synthetic workloads: library shapes, synthon tables, decoder weights, queries.

Every random value comes from a counter-based SplitMix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): value n of
stream (seed, name) is mix64(key + (n + 1) * GOLDEN) with key derived from the seed
and a hash of the stream name. Normal variates use the Box-Muller transform. The
logarithm, exponential and cosine it needs are evaluated here with series built
only from correctly rounded IEEE operations (+, -, *, /, sqrt, frexp, ldexp), so the
same seed yields bit-identical float32 inputs on any x86-64 host, whatever SIMD
variants numpy or libm pick there.

The shapes follow the paper's libraries: two- and three-component reactions whose
R-groups hold tens to thousands of synthons (Section 3.1, Appendix A.1), 28 task
heads in the paper's probe (Appendix A.8), constraint sets of two to six one- or
two-sided thresholds (Table "Constraint sets"). Values are N(0, 1) embeddings and
Xavier-uniform weights, not trained models.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

ACT_NONE, ACT_RELU, ACT_SILU = 0, 1, 2


# ----------------------------------------------------------------------------
# SplitMix64, counter based
# ----------------------------------------------------------------------------
def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _mix64_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _fnv1a(name: str) -> int:
    h = 0xCBF29CE484222325
    for ch in name.encode():
        h ^= ch
        h = (h * 0x100000001B3) & MASK64
    return h


def stream_key(seed: int, name: str) -> int:
    return _mix64_int((seed * 0x9E3779B97F4A7C15 + _fnv1a(name)) & MASK64)


def stream_u64(seed: int, name: str, n: int, offset: int = 0) -> np.ndarray:
    """Values offset .. offset+n-1 of the stream (seed, name) as uint64."""
    key = np.uint64(stream_key(seed, name))
    ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = key + ctr * GOLDEN
    return _mix64(state)


def uniform_f64(seed: int, name: str, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits."""
    x = stream_u64(seed, name, n, offset)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ----------------------------------------------------------------------------
# Deterministic elementary functions (only correctly rounded operations)
# ----------------------------------------------------------------------------
_LN2 = 0.6931471805599453  # nearest double to ln 2
_SQRT_HALF = 0.7071067811865476


def _log(x: np.ndarray) -> np.ndarray:
    """Natural log for x > 0: x = m * 2**e with m in [sqrt(1/2), sqrt(2)),
    log m = 2 * atanh(s), s = (m - 1) / (m + 1), |s| < 0.172."""
    m, e = np.frexp(x)  # m in [0.5, 1)
    small = m < _SQRT_HALF
    m = np.where(small, m * 2.0, m)
    e = np.where(small, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    acc = np.zeros_like(s)
    for n in range(25, 0, -2):  # odd terms 1/25 ... 1/1, Horner in s^2
        acc = acc * s2 + 1.0 / n
    return 2.0 * s * acc + e * _LN2


def _exp(x: np.ndarray) -> np.ndarray:
    """exp(x) = 2**k * exp(r), k = round(x / ln 2), |r| <= ln(2)/2; Taylor to r^20."""
    k = np.round(x / _LN2)
    r = x - k * _LN2
    acc = np.ones_like(r)
    for n in range(20, 0, -1):
        acc = 1.0 + acc * r / n
    return np.ldexp(acc, k.astype(np.int64))


def _sin_cos_small(a: np.ndarray):
    """sin and cos of |a| <= pi/4 by Taylor series (terms to a^21)."""
    a2 = a * a
    s = np.zeros_like(a)
    c = np.zeros_like(a)
    # sin: a - a^3/3! + ... ; cos: 1 - a^2/2! + ...
    term_s = a.copy()
    term_c = np.ones_like(a)
    for n in range(0, 11):
        s = s + term_s
        c = c + term_c
        term_s = -term_s * a2 / ((2 * n + 2) * (2 * n + 3))
        term_c = -term_c * a2 / ((2 * n + 1) * (2 * n + 2))
    return s, c


def _cos_2pi(v: np.ndarray) -> np.ndarray:
    """cos(2*pi*v) for v in [0, 1): reduce to an octant with exact steps."""
    w = v * 8.0  # exact (power of two)
    octant = np.floor(w)
    f = w - octant  # exact, in [0, 1)
    o = octant.astype(np.int64) & 7
    quarter_pi = math.pi / 4.0
    # within octant o the angle is (o + f) * pi/4
    a = np.where((o & 1) == 1, (1.0 - f), f) * quarter_pi
    s, c = _sin_cos_small(a)
    # angle theta = o*pi/4 + f*pi/4. For odd octants we evaluated at the
    # mirrored angle (1-f)*pi/4 measured from the next multiple of pi/2 ... map:
    # o=0: cos(a)      o=1: sin(a)      o=2: -sin(a)     o=3: -cos(a)
    # o=4: -cos(a)     o=5: -sin(a)     o=6: sin(a)      o=7: cos(a)
    out = np.select(
        [o == 0, o == 1, o == 2, o == 3, o == 4, o == 5, o == 6, o == 7],
        [c, s, -s, -c, -c, -s, s, c],
    )
    return out


def normal_f64(seed: int, name: str, n: int, offset: int = 0) -> np.ndarray:
    """N(0, 1) by Box-Muller on counters (2i, 2i+1), cosine branch."""
    u = uniform_f64(seed, name, 2 * n, 2 * offset).reshape(n, 2)
    u1 = 1.0 - u[:, 0]  # (0, 1]
    r = np.sqrt(-2.0 * _log(u1))
    return r * _cos_2pi(u[:, 1])


_NATIVE = None
_NATIVE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgen_native.so")


def build_native() -> str:
    """Compile the bulk generator (gen_native.c) next to this file."""
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen_native.c")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", src, "-o", _NATIVE_PATH, "-lm"])
    return _NATIVE_PATH


def _native():
    global _NATIVE
    if _NATIVE is None and os.path.exists(_NATIVE_PATH):
        lib = ctypes.CDLL(_NATIVE_PATH)
        lib.gen_normal_f32.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_void_p]
        lib.gen_normal_f32.restype = None
        _NATIVE = lib
    return _NATIVE


def normal_f32(seed: int, name: str, n: int, offset: int = 0, native: bool = True) -> np.ndarray:
    """float32 N(0, 1) values; the compiled generator, when built, gives the same bits."""
    lib = _native() if native else None
    if lib is None:
        return normal_f64(seed, name, n, offset).astype(np.float32)
    out = np.empty(n, dtype=np.float32)
    lib.gen_normal_f32(stream_key(seed, name), offset, n, out.ctypes.data)
    return out


def uniform_sym_f32(seed: int, name: str, n: int, bound: float) -> np.ndarray:
    """U(-bound, bound) rounded to float32."""
    u = uniform_f64(seed, name, n)
    return ((2.0 * u - 1.0) * bound).astype(np.float32)


# ----------------------------------------------------------------------------
# Library, decoder and query containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Library:
    """A combinatorial synthesis library: reactions, their R-groups (slots) and
    one embedding row per (reaction, slot, synthon), rows in that order.
    (Section 4.2: D = (T, R, S, psi, phi); Appendix A.1.)"""

    n_slots: np.ndarray  # uint32 [T], 2 or 3
    slot_sizes: np.ndarray  # uint32 [sum n_slots]
    d: int
    tables: np.ndarray  # float32 [rows, d]

    @property
    def n_reactions(self) -> int:
        return int(len(self.n_slots))

    def reaction_counts(self) -> List[int]:
        out, p = [], 0
        for t in range(self.n_reactions):
            c = 1
            for s in range(int(self.n_slots[t])):
                c *= int(self.slot_sizes[p + s])
            out.append(c)
            p += int(self.n_slots[t])
        return out

    @property
    def n_compounds(self) -> int:
        return sum(self.reaction_counts())

    @property
    def n_rows(self) -> int:
        return int(self.slot_sizes.sum())


@dataclasses.dataclass
class Decoder:
    """Decoder weights: W[l] is dims[l+1] x dims[l] row-major, b[l] has dims[l+1]
    entries; the activation follows every layer but the last."""

    dims: List[int]
    act: int
    W: List[np.ndarray]
    b: List[np.ndarray]

    @property
    def n_layers(self) -> int:
        return len(self.W)

    @property
    def n_heads(self) -> int:
        return self.dims[-1]


@dataclasses.dataclass
class Constraint:
    head: int
    lo: float  # float32 value, -inf for one-sided upper bounds
    hi: float  # float32 value, +inf for one-sided lower bounds


@dataclasses.dataclass
class Query:
    """Objective weights over heads (maximise w . heads), inclusive bounds
    lo <= head <= hi, top-k size, and an optional reaction subset."""

    w: np.ndarray  # float32 [H]
    constraints: List[Constraint]
    k: int
    reactions: Optional[Sequence[int]] = None
    keep_violators: bool = False  # fill the answer with the least-violating compounds


# ----------------------------------------------------------------------------
# Builders
# ----------------------------------------------------------------------------
def make_library(seed: int, n_slots: Sequence[int], slot_sizes: Sequence[int], d: int,
                 stream: str = "tables") -> Library:
    n_slots = np.asarray(n_slots, dtype=np.uint32)
    slot_sizes = np.asarray(slot_sizes, dtype=np.uint32)
    assert slot_sizes.size == int(n_slots.sum())
    rows = int(slot_sizes.sum())
    tables = normal_f32(seed, stream, rows * d).reshape(rows, d)
    return Library(n_slots=n_slots, slot_sizes=slot_sizes, d=d, tables=tables)


def make_factorizer(seed: int, slot_sizes: Sequence[int], d: int, d_u: int):
    """Synthetic inputs of the associative embeddings (Section 4.2): one key
    matrix K_r (d x d_u, entries N(0, 1/d_u)) per R-group and one value vector
    (d_u, N(0, 1)) per table row. Returns (keys [R, d, d_u], values [rows, d_u])."""
    n_r, rows = len(slot_sizes), int(np.sum(slot_sizes))
    keys = (normal_f32(seed, "assoc_keys", n_r * d * d_u) * np.float32(1.0 / math.sqrt(d_u))).reshape(n_r, d, d_u)
    values = normal_f32(seed, "assoc_values", rows * d_u).reshape(rows, d_u)
    return keys.astype(np.float32), values


def make_decoder(seed: int, dims: Sequence[int], act: int) -> Decoder:
    """Xavier-uniform weights U(+-sqrt(6/(fan_in+fan_out))), biases U(+-1/sqrt(fan_in))."""
    W, b = [], []
    for l in range(len(dims) - 1):
        fi, fo = int(dims[l]), int(dims[l + 1])
        a = math.sqrt(6.0 / (fi + fo))
        W.append(uniform_sym_f32(seed, f"W{l}", fo * fi, a).reshape(fo, fi))
        b.append(uniform_sym_f32(seed, f"b{l}", fo, 1.0 / math.sqrt(fi)))
    return Decoder(dims=[int(x) for x in dims], act=act, W=W, b=b)


def lognormal_counts(seed: int, name: str, n: int, median: float, sigma: float,
                     lo: int, hi: int) -> np.ndarray:
    z = normal_f64(seed, name, n)
    v = _exp(math.log(median) + sigma * z)
    return np.clip(np.floor(v + 0.5), lo, hi).astype(np.int64)


def _cap_total(n_slots: List[int], sizes: List[List[int]], target: int, floor: int) -> None:
    """Shrink the largest slot of the largest reaction by 10% (not below floor)
    until the compound total is at most target."""
    def count(t):
        c = 1
        for x in sizes[t]:
            c *= x
        return c

    total = sum(count(t) for t in range(len(sizes)))
    while total > target:
        t = max(range(len(sizes)), key=lambda i: (count(i), -i))
        s = max(range(len(sizes[t])), key=lambda j: (sizes[t][j], -j))
        old = count(t)
        new_size = max(floor, int(sizes[t][s] * 0.9))
        if new_size == sizes[t][s]:
            break
        sizes[t][s] = new_size
        total += count(t) - old


def library_shapes_c1(seed: int = 1):
    """40 reactions (28 two-slot, 12 three-slot), per-slot counts lognormal with
    median 150 in [20, 3000], capped to about 1.04e7 compounds."""
    T, n3 = 40, 12
    order = np.argsort(uniform_f64(seed, "three_slot_pick", T), kind="stable")
    three = set(int(i) for i in order[:n3])
    n_slots = [3 if t in three else 2 for t in range(T)]
    raw = lognormal_counts(seed, "slot_counts", sum(n_slots), 150.0, 1.0, 20, 3000)
    sizes, p = [], 0
    for t in range(T):
        sizes.append([int(x) for x in raw[p:p + n_slots[t]]])
        p += n_slots[t]
    _cap_total(n_slots, sizes, 10_400_000, 20)
    flat = [x for s in sizes for x in s]
    return n_slots, flat


def library_shapes_probe(seed: int, target: int, T: int = 40, n3: int = 12):
    """The benchmark library recipe (T reactions, n3 of them three-slot, per-slot
    counts lognormal with median 150 in [20, 3000]) capped to about `target`
    compounds."""
    order = np.argsort(uniform_f64(seed, "three_slot_pick", T), kind="stable")
    three = set(int(i) for i in order[:n3])
    n_slots = [3 if t in three else 2 for t in range(T)]
    raw = lognormal_counts(seed, "slot_counts", sum(n_slots), 150.0, 1.0, 20, 3000)
    sizes, p = [], 0
    for t in range(T):
        sizes.append([int(x) for x in raw[p:p + n_slots[t]]])
        p += n_slots[t]
    _cap_total(n_slots, sizes, target, 20)
    return n_slots, [x for s in sizes for x in s]


def config_probe(seed: int, n_slots, sizes, d: int = 64, n_heads: int = 28):
    """A library of the given shape with the paper's surrogate head: embedding
    width d = 64 and a LinearProbe of 28 linear heads (Section 5.1 and Appendix
    A.8), Xavier weights from the seed."""
    lib = make_library(seed, n_slots, sizes, d)
    dec = make_decoder(seed, [d, n_heads], ACT_NONE)
    return lib, dec


def probe_query(seed: int, head_quantile, k: int, target: int = 0, n_heads: int = 28, lipinski: bool = True):
    """The runtime table's query (Section 5.2, Table tab:runtime): minimise the
    docking score of one target (heads 0..4 stand for the five targets; w = -1)
    under the four Lipinski bounds (Appendix A.7, Table tab:constraints: four
    upper bounds), here on four seeded property heads (5..n_heads-1), each at a
    seeded quantile in [0.6, 0.9] of the head's distribution
    (`head_quantile(head, q)`)."""
    w = np.zeros(n_heads, dtype=np.float32)
    w[target] = -1.0
    cons = []
    if lipinski:
        props = list(range(5, n_heads))
        perm = np.argsort(uniform_f64(seed, "probe_heads", len(props)), kind="stable")
        quant = 0.6 + 0.3 * uniform_f64(seed, "probe_quant", 4)
        for i in range(4):
            h = props[int(perm[i])]
            cons.append(Constraint(h, -math.inf, float(np.float32(head_quantile(h, float(quant[i]))))))
    return Query(w=w, constraints=cons, k=k)


def config_c0():
    """Tiny FP32 case: 1 reaction, 2 slots x 300 synthons, d=64, MLP 64->128 (ReLU)->5;
    maximise head 0 with head1 <= 0.5 and head2 >= -0.5, k = 100."""
    lib = make_library(0, [2], [300, 300], 64)
    dec = make_decoder(0, [64, 128, 5], ACT_RELU)
    w = np.zeros(5, dtype=np.float32)
    w[0] = 1.0
    q = Query(w=w, constraints=[Constraint(1, -math.inf, 0.5), Constraint(2, -0.5, math.inf)], k=100)
    return lib, dec, q


def config_c1_model(seed: int = 1):
    n_slots, sizes = library_shapes_c1(seed)
    lib = make_library(seed, n_slots, sizes, 256)
    dec = make_decoder(seed, [256, 512, 512, 15], ACT_SILU)
    return lib, dec


def config_c1(seed: int = 1):
    """Benchmark-shaped case (about 1.04e7 compounds): the library and decoder.
    Query thresholds need head quantiles and are stored beside the tests."""
    return config_c1_model(seed)


def config_c3_shape(seed: int = 2, target: float = 3e10):
    """2,000 reactions with 2 or 3 slots, per-slot counts lognormal (median 800,
    at most 10,000). The number of three-slot reactions is the smallest that
    reaches `target` compounds (3e10 for the large case); the largest reactions
    are then trimmed to at most the target. Returns (n_slots, sizes)."""
    T = 2000
    raw = lognormal_counts(seed, "slot_counts", 3 * T, 800.0, 1.0, 20, 10_000)
    pick = uniform_f64(seed, "three_slot_pick", T)
    order = np.argsort(pick, kind="stable")
    n3 = T
    for m in range(0, T + 1):
        three = set(int(i) for i in order[:m])
        total = 0
        for t in range(T):
            a, b, c = (int(x) for x in raw[3 * t:3 * t + 3])
            total += a * b * c if t in three else a * b
        if total >= target:
            n3 = m
            break
    three = set(int(i) for i in order[:n3])
    n_slots, sizes = [], []
    for t in range(T):
        ns = 3 if t in three else 2
        n_slots.append(ns)
        sizes.append([int(x) for x in raw[3 * t:3 * t + ns]])
    _cap_total(n_slots, sizes, int(target), 20)
    sizes = [x for s in sizes for x in s]
    return n_slots, sizes


def seeded_query_c1(seed: int, n_heads: int = 15):
    """Seeded choices for the benchmark-shaped query: the docking-like head to
    minimise (0..4), four property heads (5..14) to bound, each bound's side and
    its target quantile in [0.6, 0.9]. Threshold values are filled in later from
    head quantiles of a sample."""
    u = uniform_f64(seed, "query_c1", 16)
    obj = int(u[0] * 5)
    props = list(range(5, n_heads))
    perm = np.argsort(uniform_f64(seed, "query_c1_heads", len(props)), kind="stable")
    heads = [props[int(i)] for i in perm[:4]]
    sides = ["hi" if u[1 + i] < 0.5 else "lo" for i in range(4)]
    quant = [0.6 + 0.3 * float(u[5 + i]) for i in range(4)]
    return obj, heads, sides, quant


def sample_ids(seed: int, name: str, n_total: int, n: int) -> np.ndarray:
    """n compound ids drawn uniformly (with replacement) from [0, n_total)."""
    x = stream_u64(seed, name, n)
    return (x % np.uint64(n_total)).astype(np.uint64)


def serving_stream(seed: int, n: int, qps: float, reaction_counts: Sequence[int], size_lo: float, size_hi: float,
                   head_quantile, n_heads: int = 15, ks=(100, 1000, 10000)):
    """A seeded stream of queries for the serving loop.

    Arrivals are a Poisson process (exponential gaps, rate qps). Each query has
    objective weights N(0, 1) over the heads, 2-6 one-sided bounds on distinct
    heads at quantiles drawn from [0.6, 0.9] (values from `head_quantile(head, q)`,
    which the caller supplies), k drawn from `ks`, and a library that is a subset
    of whole reactions: a target count is drawn log-uniformly in [size_lo, size_hi],
    and reactions are added in a seeded random order until the target is reached,
    skipping any that would take the subset past size_hi (so one large reaction
    cannot carry it out of the range). Returns a list of (arrival_s, Query)."""
    u = uniform_f64(seed, "serve_u", 16 * n).reshape(n, 16)
    z = normal_f64(seed, "serve_w", n * n_heads).reshape(n, n_heads)
    gaps = -_log(1.0 - uniform_f64(seed, "serve_gap", n)) / qps
    t = np.cumsum(gaps)
    T = len(reaction_counts)
    out = []
    for i in range(n):
        order = np.argsort(uniform_f64(seed + 1000003 * (i + 1), "serve_perm", T), kind="stable")
        target = math.exp(math.log(size_lo) + (math.log(size_hi) - math.log(size_lo)) * float(u[i, 0]))
        subset, tot = [], 0
        for r in order:
            c = int(reaction_counts[int(r)])
            if tot + c > size_hi:
                continue
            subset.append(int(r))
            tot += c
            if tot >= target:
                break
        if not subset:  # every reaction is larger than size_hi: the smallest one
            subset = [int(np.argmin(np.asarray(reaction_counts)))]
        n_thr = 2 + int(u[i, 1] * 5)
        heads = np.argsort(uniform_f64(seed + 7919 * (i + 1), "serve_heads", n_heads), kind="stable")[:n_thr]
        cons = []
        for j, h in enumerate(heads):
            q = 0.6 + 0.3 * float(u[i, 2 + j])
            if u[i, 8 + j] < 0.5:
                cons.append(Constraint(int(h), -math.inf, float(np.float32(head_quantile(int(h), q)))))
            else:
                cons.append(Constraint(int(h), float(np.float32(head_quantile(int(h), 1.0 - q))), math.inf))
        k = int(ks[min(len(ks) - 1, int(u[i, 14] * len(ks)))])
        out.append((float(t[i]), Query(w=z[i].astype(np.float32), constraints=cons, k=k,
                                       reactions=sorted(subset))))
    return out


def config_c3(seed: int = 2):
    """The large streamed case: the C3 shape (about 2.9e10 compounds, 5.3M rows),
    d = 256, decoder 256 -> 512 -> 512 (SiLU) -> 15. The tables take 5.4 GB."""
    n_slots, sizes = config_c3_shape(seed)
    lib = make_library(seed, n_slots, sizes, 256)
    dec = make_decoder(seed, [256, 512, 512, 15], ACT_SILU)
    return lib, dec
