"""Device-level checks of the two worklist filters of Section 4, read back
through sx_run_iterations / sx_frontier_get:

  - the paper's worked example (Fig. back-sample-sssp, Section 4): the online
    filter turns active {b, d} into the list {e, c}; the ballot filter after
    iteration 3 gives the words 0100 (a-d) and 01111 (e-i) and the sorted list
    {b, f, g, h, i}  (tests/golden/sssp_worked_example.txt);
  - BFS on R-MAT and grid graphs: after every level t, the online list is the
    set of vertices the oracle puts at depth t + 1, each exactly once (one
    successful claim per vertex), and the ballot list is that set sorted and
    unique in every bin, with ballot words whose set bits are exactly it."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
import paper_1812_04070_amd as sx
from paper_1812_04070_amd import gen
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def engine():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = sx.Engine(0)
    yield e
    e.close()


def _golden():
    edges, w, facts = [], [], {}
    names = "abcdefghi"
    for line in open(os.path.join(HERE, "golden", "sssp_worked_example.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "e":
            edges.append((names.index(tok[1]), names.index(tok[2])))
            w.append(int(tok[3]))
        else:
            facts[tok[0]] = tok[1:]
    return gen.from_edges(9, edges, w, name="worked-example"), facts, names


def _frontier(engine, dg, algo, src, iters, policy, cap, nwords=0):
    import torch
    out = torch.empty(max(dg.n, 1), dtype=torch.int32, device=engine.device)
    p = engine.program(algo)
    sx.sx_program_set_policy(p, policy.c())
    sx.sx_run_iterations(p, dg.handle, src, out.data_ptr(), iters, engine.stream())
    return sx.sx_frontier_get(dg.handle, cap, nwords, engine.stream())


def test_worked_example_online_list(engine):
    g, facts, names = _golden()
    dg = engine.load(g)
    announce("worked example: online list after iteration 2")
    pol = sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_ONLINE)
    v, b, from_ballot, _ = _frontier(engine, dg, sx.SX_SSSP, 0, 2, pol, 64)
    assert not from_ballot
    # the online filter appends in order of arrival: compare as a multiset
    assert sorted(names[x] for x in v) == sorted(facts["iter2_next"])
    dg.close()


def test_worked_example_ballot_words(engine):
    g, facts, names = _golden()
    dg = engine.load(g)
    announce("worked example: ballot filter after iteration 3")
    pol = sx.Policy(direction=sx.SX_DIR_PUSH, filter=sx.SX_FILTER_BALLOT)
    v, b, from_ballot, words = _frontier(engine, dg, sx.SX_SSSP, 0, 3, pol, 64, nwords=1)
    assert from_ballot
    assert [names[x] for x in v] == facts["iter3_next"]          # sorted, unique
    bits = "".join(str((int(words[0]) >> i) & 1) for i in range(9))
    assert bits[0:4] == facts["ballot_word_a_d"][0]
    assert bits[4:9] == facts["ballot_word_e_i"][0]
    dg.close()


@pytest.mark.parametrize("name,make", [
    ("rmat12", lambda: gen.rmat(12, seed=6, weights=(1, 64))),
    ("rmat14", lambda: gen.rmat(14, seed=8, weights=(1, 64))),
    ("grid-60", lambda: gen.grid(60, 0.1, seed=3, weights=(1, 64))),
])
def test_bfs_lists_per_level(engine, name, make):
    g = make()
    src = gen.max_degree_vertex(g)
    depth = oracle.bfs_g(g, src)
    levels = int(depth.max())
    dg = engine.load(g)
    nwords = (g.n + 63) // 64
    deg = g.out_degree()
    for t in range(1, min(levels, 40) + 1):
        expect = np.nonzero(depth == t)[0]
        announce(f"filters {name} level {t}: {expect.size} vertices")
        for filt in (sx.SX_FILTER_ONLINE, sx.SX_FILTER_BALLOT):
            pol = sx.Policy(direction=sx.SX_DIR_PUSH, filter=filt, bin_small=16, bin_large=128)
            v, b, from_ballot, words = _frontier(engine, dg, sx.SX_BFS, src, t, pol, g.n + 64, nwords)
            # every vertex of the level exactly once (no duplicates)
            assert v.size == expect.size and np.array_equal(np.sort(v), expect), (name, t, filt)
            # each entry sits in the bin of its degree
            want = np.where(deg[v] < 16, 0, np.where(deg[v] < 128, 1, 2))
            assert np.array_equal(b, want)
            if filt == sx.SX_FILTER_BALLOT:
                assert from_ballot
                for k in range(3):
                    part = v[b == k]
                    assert np.all(np.diff(part) > 0), "ballot list not sorted and unique"
                flagged = np.nonzero(np.unpackbits(words.view(np.uint8), bitorder="little")[:g.n])[0]
                assert np.array_equal(flagged, expect)
            else:
                assert not from_ballot
    dg.close()


def test_sssp_online_list_has_no_duplicates(engine):
    """An SSSP vertex lowered several times in one iteration enters the next
    list once (its stamp is exchanged by the first success)."""
    g = gen.rmat(13, seed=12, weights=(1, 64))
    src = gen.max_degree_vertex(g)
    dg = engine.load(g)
    for t in (1, 2, 3):
        announce(f"sssp online list iteration {t}")
        v, b, fb, _ = _frontier(engine, dg, sx.SX_SSSP, src, t, sx.Policy(direction=sx.SX_DIR_PUSH,
                                                                           filter=sx.SX_FILTER_ONLINE),
                                g.n + 64)
        assert not fb and v.size > 0
        assert np.unique(v).size == v.size
    dg.close()
