"""Input generator: RNG test vectors, lattices and CZ patterns."""

import numpy as np

import synth
from synth import SplitMix64


def test_splitmix64_published_vectors():
    # First outputs of SplitMix64 seeded with 0 (reference outputs of the
    # published generator).
    r = SplitMix64(0)
    assert [r.next() for _ in range(4)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_uniform_and_bits_are_from_top_bits():
    a, b = SplitMix64(9), SplitMix64(9)
    for _ in range(100):
        u = a.uniform()
        z = b.next()
        assert 0.0 <= u < 1.0 and u == (z >> 11) / 2.0 ** 53


def _all_couplers(lat):
    out = set()
    for (r, c) in lat.sites:
        for (dr, dc) in ((0, 1), (1, 0)):
            if (r + dr, c + dc) in lat.qid:
                out.add((lat.qid[(r, c)], lat.qid[(r + dr, c + dc)]))
    return out


def test_patterns_partition_couplers_into_matchings():
    for lat in (synth.grid(4, 4), synth.grid(5, 5), synth.grid(7, 7), synth.diamond70()):
        pats = synth.cz_patterns(lat)
        assert len(pats) == 8
        seen = []
        for p in pats:
            qs = [q for e in p for q in e]
            assert len(qs) == len(set(qs)), "pattern is not a matching"
            seen += p
        assert len(seen) == len(set(seen))
        assert set(seen) == _all_couplers(lat)


def test_diamond70_shape():
    lat = synth.diamond70()
    assert lat.n == 70
    assert sum(len(p) for p in synth.cz_patterns(lat)) == 123
    assert (0, 0) not in lat.qid and (7, 8) not in lat.qid


def test_circuit_layout_uniform_rule():
    lat = synth.grid(4, 4)
    circ = synth.random_circuit(lat, 10, 101)
    n = lat.n
    assert (circ[:n, 0] == synth.GATE_H).all() and (circ[-n:, 0] == synth.GATE_H).all()
    pats = synth.cz_patterns(lat)
    for t in range(1, 11):
        cyc = circ[circ[:, 3] == t]
        cz = {(int(a), int(b)) for k, a, b, _ in cyc if k == synth.GATE_CZ}
        assert cz == set(pats[(t - 1) % 8])
        busy = {q for e in cz for q in e}
        one = [int(a) for k, a, _, _ in cyc if k != synth.GATE_CZ]
        assert sorted(one) == [q for q in range(n) if q not in busy]


def test_circuit_paper_rule():
    lat = synth.grid(4, 4)
    circ = synth.random_circuit(lat, 12, 7, rule="paper")
    n = lat.n
    prev_cz = set()
    prev_1q = set(range(n))
    for t in range(1, 13):
        cyc = circ[circ[:, 3] == t]
        cz = {q for k, a, b, _ in cyc if k == synth.GATE_CZ for q in (int(a), int(b))}
        for k, a, _, _ in cyc:
            if k == synth.GATE_CZ:
                continue
            a = int(a)
            if a in prev_cz:
                assert k in (synth.GATE_SQRT_X, synth.GATE_SQRT_Y)
            else:
                assert a in prev_1q and k == synth.GATE_T
        got = {int(a) for k, a, _, _ in cyc if k != synth.GATE_CZ}
        assert got == {q for q in range(n) if q not in cz and (q in prev_cz or q in prev_1q)}
        prev_1q = {int(a) for k, a, _, _ in cyc if k in (synth.GATE_SQRT_X, synth.GATE_SQRT_Y)}
        prev_cz = cz


def test_bitstrings_and_slices_deterministic():
    a = synth.random_bitstrings(25, 64, 202)
    b = synth.random_bitstrings(25, 64, 202)
    assert a.dtype == np.uint8 and a.shape == (64, 25) and (a == b).all()
    assert set(np.unique(a)) <= {0, 1}
    s = synth.random_slices(16, 32, 303)
    assert s.dtype == np.uint64 and (s < 2 ** 16).all()


def test_request_mix():
    reqs = synth.request_mix(16)
    assert len(reqs) == 16
    for r in reqs:
        assert r["family"] in synth.circuits.REQUEST_FAMILIES
        assert r["bitstring"].shape == (r["lattice"].n,)
