"""Random 2D-lattice circuits in the style of the paper's benchmark (Section
"Benchmarking and the Experimental Setup", the enumerated circuit
prescription), drawn from SplitMix64.

A circuit is an int32 array of shape [n_gates, 4] with rows
(kind, q0, q1, moment) in application order; q1 = -1 for one-qubit gates.
Qubits are numbered row-major over the lattice sites that are present.

Two single-qubit rules are provided:

* ``"uniform"`` (default, used by the measured workloads): in every middle
  cycle each qubit not touched by a CZ receives one gate drawn uniformly from
  (sqrt X, sqrt Y, T).
* ``"paper"``: the rule of the prescription's item 3 -- a qubit idle in cycle
  t receives a gate drawn uniformly from (sqrt X, sqrt Y) if it was in a CZ in
  cycle t-1, else a T if it received sqrt X, sqrt Y or H in the previous
  layer, else nothing.  The previous layer of cycle 1 is the H layer.

The eight CZ configurations are this project's own definition (the paper does
not spell them out): with sites (r, c),
H(a,b) = {(r,c)-(r,c+1) : c = a, r = b (mod 2)} and
V(a,b) = {(r,c)-(r+1,c) : r = a, c = b (mod 2)}, used in the order
H(0,0) H(1,1) V(0,0) V(1,1) H(0,1) H(1,0) V(0,1) V(1,0); cycle t (1-based)
uses pattern (t-1) mod 8.  Each pattern is a matching and together they cover
every nearest-neighbour coupler once.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .rng import SplitMix64

GATE_H = 0
GATE_SQRT_X = 1
GATE_SQRT_Y = 2
GATE_T = 3
GATE_CZ = 4
GATE_NAMES = {GATE_H: "H", GATE_SQRT_X: "sqrtX", GATE_SQRT_Y: "sqrtY",
              GATE_T: "T", GATE_CZ: "CZ"}


@dataclass
class Lattice:
    rows: int
    cols: int
    sites: list  # (r, c) present, row-major
    qid: dict = field(default_factory=dict)  # (r, c) -> qubit id
    cut: frozenset = frozenset()  # couplers absent between adjacent present sites, ((r, c), (r', c'))

    @property
    def n(self) -> int:
        return len(self.sites)


def _lattice(rows: int, cols: int, removed=(), cut=()) -> Lattice:
    removed = set(removed)
    sites = [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in removed]
    return Lattice(rows, cols, sites, {s: i for i, s in enumerate(sites)},
                   frozenset(tuple(sorted(pair)) for pair in cut))


def grid(rows: int, cols: int) -> Lattice:
    return _lattice(rows, cols)


def diamond70() -> Lattice:
    """70-qubit lattice: an 8x9 square grid (a diamond when drawn at 45
    degrees) without its two corner sites (0,0) and (7,8); 123 couplers."""
    return _lattice(8, 9, removed=[(0, 0), (7, 8)])


def diamond72() -> Lattice:
    """72-qubit lattice with two degree-1 qubits: the full 8x9 grid whose
    corner sites (0,0) and (7,8) keep one coupler each, to (0,1) and (7,7)
    (the couplers (0,0)-(1,0) and (6,8)-(7,8) are absent): the 70-qubit
    lattice plus two qubits whose only neighbour is on it; 125 couplers."""
    return _lattice(8, 9, cut=[((0, 0), (1, 0)), ((6, 8), (7, 8))])


def cz_patterns(lat: Lattice):
    """The eight coupler patterns, each a list of (q0, q1) with q0 < q1."""
    def hpat(a, b):
        out = []
        for (r, c) in lat.sites:
            if c % 2 == a and r % 2 == b and (r, c + 1) in lat.qid and ((r, c), (r, c + 1)) not in lat.cut:
                out.append((lat.qid[(r, c)], lat.qid[(r, c + 1)]))
        return out

    def vpat(a, b):
        out = []
        for (r, c) in lat.sites:
            if r % 2 == a and c % 2 == b and (r + 1, c) in lat.qid and ((r, c), (r + 1, c)) not in lat.cut:
                out.append((lat.qid[(r, c)], lat.qid[(r + 1, c)]))
        return out

    return [hpat(0, 0), hpat(1, 1), vpat(0, 0), vpat(1, 1),
            hpat(0, 1), hpat(1, 0), vpat(0, 1), vpat(1, 0)]


def random_circuit(lat: Lattice, depth: int, seed: int, rule: str = "uniform",
                   final_h: bool = True, single_qubit: bool = True,
                   gate_set=(GATE_SQRT_X, GATE_SQRT_Y, GATE_T)) -> np.ndarray:
    """Circuit 1 + depth + 1 on ``lat``.  ``gate_set`` (uniform rule only)
    lists the gates drawn from, in draw order; index = floor(len * u)."""
    if rule not in ("uniform", "paper"):
        raise ValueError(f"unknown rule {rule!r}")
    rng = SplitMix64(seed)
    pats = cz_patterns(lat)
    n = lat.n
    rows = [(GATE_H, q, -1, 0) for q in range(n)]
    prev_cz = [False] * n
    prev_1q = [True] * n  # the H layer counts as the previous layer of cycle 1
    for t in range(1, depth + 1):
        pat = pats[(t - 1) % 8]
        busy = [False] * n
        for (a, b) in pat:
            rows.append((GATE_CZ, a, b, t))
            busy[a] = busy[b] = True
        got_1q = [False] * n
        if single_qubit:
            for q in range(n):
                if busy[q]:
                    continue
                if rule == "uniform":
                    g = gate_set[int(len(gate_set) * rng.uniform())]
                else:
                    if prev_cz[q]:
                        g = (GATE_SQRT_X, GATE_SQRT_Y)[int(2 * rng.uniform())]
                    elif prev_1q[q]:
                        g = GATE_T
                    else:
                        continue
                rows.append((g, q, -1, t))
                got_1q[q] = g in (GATE_SQRT_X, GATE_SQRT_Y, GATE_H)
        prev_cz, prev_1q = busy, got_1q
    if final_h:
        rows += [(GATE_H, q, -1, depth + 1) for q in range(n)]
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def random_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    """uint8 array [count, n_qubits]; bit = next() >> 63, row by row."""
    rng = SplitMix64(seed)
    out = np.empty((count, n_qubits), dtype=np.uint8)
    for i in range(count):
        for q in range(n_qubits):
            out[i, q] = rng.bit()
    return out


def random_slices(log2_slices: int, count: int, seed: int) -> np.ndarray:
    """uint64 slice ids drawn as next() mod 2^k."""
    rng = SplitMix64(seed)
    mod = 1 << log2_slices
    return np.asarray([rng.below(mod) for _ in range(count)], dtype=np.uint64)


# Workloads.  Seeds: circuit = seed, bitstrings = seed + 1, sampled slices =
# seed + 2, request mix = seed + 3 (per-request slice counts: seed + 4).
# trials / plan_seed: restarts and seed of the order search that every
# measurement and parity test of the workload uses; chunk: slices in flight
# per call where the workload is timed on a slice range.
CONFIGS = {
    "c1": dict(name="grid4x4_d10", lattice=(4, 4), depth=10, seed=101,
               n_bitstrings=1, log2_slices=0, trials=8, plan_seed=1),
    # quick: the greedy order alone -- this workload runs all its slices in
    # flight in one fused work item, where the greedy tree costs 2.5x fewer
    # flops than the one refined for the cost of a single slice.
    "c2": dict(name="grid5x5_d16", lattice=(5, 5), depth=16, seed=201,
               n_bitstrings=64, log2_slices=6, trials=8, plan_seed=1, quick=True),
    "c3": dict(name="grid7x7_d24", lattice=(7, 7), depth=24, seed=301,
               n_bitstrings=1, log2_slices=16, log2_cap=30, n_sampled=32, trials=8, plan_seed=1),
    "c4": dict(name="diamond70_d32", lattice="diamond70", depth=32, seed=401,
               n_bitstrings=1, log2_slices=20, log2_cap=30, trials=256, plan_seed=1, chunk=64),
    # The same circuit with the outputs of its last n_open qubits left open:
    # each contraction gives the 2^n_open amplitudes of the bitstrings that
    # differ from the drawn one only there.
    "c4o": dict(name="diamond70_d32_open16", lattice="diamond70", depth=32, seed=401,
                n_bitstrings=1, log2_slices=20, log2_cap=30, trials=256, plan_seed=1, chunk=32, n_open=16),
}


def config(key: str):
    """(lattice, circuit, bitstrings, spec dict) for a named workload; a
    workload with open outputs also gets spec["open_qubits"]."""
    spec = dict(CONFIGS[key])
    lat = {"diamond70": diamond70, "diamond72": diamond72}[spec["lattice"]]() if isinstance(spec["lattice"], str) \
        else grid(*spec["lattice"])
    if spec.get("n_open"):
        spec["open_qubits"] = list(range(lat.n - spec["n_open"], lat.n))
    circ = random_circuit(lat, spec["depth"], spec["seed"])
    bs = random_bitstrings(lat.n, spec["n_bitstrings"], spec["seed"] + 1)
    return lat, circ, bs, spec


REQUEST_FAMILIES = ((4, 4, 12), (5, 5, 16), (6, 6, 20), (7, 7, 24))


REQUEST_MAX_LOG2_SLICES = 12


def request_mix(count: int = 256, seed: int = 501):
    """Uneven batch of amplitude requests: for each request a family drawn
    uniformly (floor(4u) on stream seed + 3), then a 32-bit circuit seed from
    the same stream; the request's bitstring comes from circuit seed + 1.
    Each request also asks for 2^k slices, k drawn uniformly from
    0..REQUEST_MAX_LOG2_SLICES (floor(13u) on stream seed + 4), the planner
    slicing further where a size cap demands it."""
    rng = SplitMix64(seed + 3)
    rng_k = SplitMix64(seed + 4)
    reqs = []
    for _ in range(count):
        fam = REQUEST_FAMILIES[int(len(REQUEST_FAMILIES) * rng.uniform())]
        cseed = rng.next() & 0xFFFFFFFF
        k = int((REQUEST_MAX_LOG2_SLICES + 1) * rng_k.uniform())
        lat = grid(fam[0], fam[1])
        circ = random_circuit(lat, fam[2], cseed)
        bs = random_bitstrings(lat.n, 1, cseed + 1)
        reqs.append(dict(family=fam, seed=cseed, lattice=lat, circuit=circ, bitstring=bs[0], log2_slices=k))
    return reqs
