"""The large workload itself (RMAT scale 20, 200,000,000 entries, 15-vertex
binary tree, k = 15) in the benchmark's configuration: properties that hold
at any size, since the oracle cannot run it.
- The exact colourful count is alpha = 128 times the number of colourful
  copies, so the U64 count (exact modulo 2^64, and 2^7 divides 2^64) is a
  multiple of 128.
- The vertex renumbering does not change the U64 count.
- FP32 with per-column exponents is within 1e-5 of FP64."""
import sys

import pytest

import graphgen as gg
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rmat20():
    say("large: generating RMAT scale 20")
    return gg.rmat20()


def test_large_workload_properties(rmat20):
    G = rmat20
    par, k, seed = gg.BINTREE15, 15, 5
    p = sg.Plan(par, k)
    assert p.info().alpha == 128
    g1 = sg.Graph.from_csr(G, relabel=True)
    c1 = sg.Colorings(g1, k, seed, 1, first=7)
    say("large: u64 (renumbered)")
    u1 = sg.count(p, g1, c1, "u64")
    assert int(u1["colorful_u64"][0]) % 128 == 0
    say("large: fp32s and fp64 (renumbered)")
    f32 = sg.count(p, g1, c1, "fp32s")["colorful"][0]
    f64 = sg.count(p, g1, c1, "fp64")["colorful"][0]
    assert f64 > 0 and abs(f32 - f64) <= 1e-5 * f64
    del g1, c1
    g0 = sg.Graph.from_csr(G)
    c0 = sg.Colorings(g0, k, seed, 1, first=7)
    say("large: u64 (caller order)")
    u0 = sg.count(p, g0, c0, "u64")
    assert int(u0["colorful_u64"][0]) == int(u1["colorful_u64"][0])
