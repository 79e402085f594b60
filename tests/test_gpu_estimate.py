"""(eps, delta) driver (Alg. 1's N = O(e^k log(1/delta) / eps^2), median of
means) on graphs small enough for brute force to give emb(T, G): the number
of colourings follows the stated bound, the median of means is within eps of
the exact count, the interval covers it, and the adaptive stop ends early."""
import math
import sys

import pytest

import graphgen as gg
import oracle as O
import paper_2009_11665_amd as sg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def exact_copies(G, par):
    _, maps, _ = O.brute(G, par)
    return maps / O.automorphisms(par)


@pytest.mark.parametrize("par,k", [([-1, 0, 1, 2], 4), ([-1, 0, 0, 0], 6)])
def test_estimate_covers_exact_count(par, k):
    G = gg.tiny_er(seed=7)
    emb = exact_copies(G, par)
    eps, delta = 0.2, 0.01
    P = O.colorful_probability(len(par), k)
    m = math.ceil(4 * (1 / P - 1) / eps ** 2)
    r = math.ceil(8 * math.log(1 / delta))
    say("estimate", par, "k", k, "emb", emb, "bound", r * m)
    res, trace = sg.estimate(sg.Plan(par, k), sg.Graph.from_csr(G), 99, eps, delta, "fp64")
    assert res.n_bound == r * m and res.groups == r and res.group_size == m
    assert res.n_colorings == r * m and not res.capped and not res.stopped_early
    assert abs(res.median_of_means - emb) <= eps * emb
    assert res.ci_low <= emb <= res.ci_high
    assert res.variance > 0 and res.std_error == pytest.approx(math.sqrt(res.variance / res.n_colorings))
    assert len(trace) == r and trace[-1] == pytest.approx(res.mean, rel=1e-12)
    # Var X <= emb^2 (1/P - 1), the bound the number of colourings rests on
    assert res.variance <= emb ** 2 * (1 / P - 1)


def test_estimate_adaptive_and_capped():
    G = gg.tiny_er(seed=7)
    par, k = [-1, 0, 1, 2, 3], 5
    emb = exact_copies(G, par)
    plan, g = sg.Plan(par, k), sg.Graph.from_csr(G)
    res, _ = sg.estimate(plan, g, 5, 0.05, 0.05, "fp32s", adaptive=True)
    say("adaptive", res.n_colorings, "of", res.n_bound, res.mean, emb)
    assert res.stopped_early and res.n_colorings < res.n_bound
    assert res.rel_half_width <= 0.05
    assert abs(res.mean - emb) <= 0.1 * emb
    cap, _ = sg.estimate(plan, g, 5, 0.05, 0.05, "fp64", max_colorings=2000)
    assert cap.capped and cap.n_colorings <= 2000
    with pytest.raises(sg.Sg2vError):
        sg.estimate(plan, g, 5, 0.0, 0.05)
