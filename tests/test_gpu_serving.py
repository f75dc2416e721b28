"""GPU tests of the serving engine: continuous batching with footprint admission.

Every request of a mixed stream completes; its results equal those of the same
request served alone (bit for bit: each shot depends only on program, theta,
seed and shot index) and agree with the oracle; energy+gradient requests equal
a direct qsv_expval_grad call.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sim

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_11599_amd import Context
    c = Context(0)
    yield c
    c.close()


def _trace(ctx, count=36, seed=7):
    rng = np.random.default_rng(seed)
    reqs = []
    vqe_prog = ctx.load(W.c4_ansatz(8, 2))
    for i in range(count):
        arrival = 0.01 * i
        if i % 5 == 4:
            coeffs, codes = W.c4_hamiltonian(seed=100 + i, n=8, terms=10)
            theta = rng.uniform(-np.pi, np.pi, 32)
            reqs.append({"id": i, "arrival": arrival, "kind": "vqe", "prog": vqe_prog, "theta": theta,
                         "coeffs": coeffs, "codes": codes})
        else:
            n = int(rng.integers(3, 17))
            src = W.c1_program(seed=200 + i, n=n, layers=int(rng.integers(2, 8)),
                               sites=tuple(sorted(rng.choice(np.arange(1, 3), size=int(rng.integers(0, 3)),
                                                             replace=False))))
            reqs.append({"id": i, "arrival": arrival, "kind": "shots", "src": src, "prog": ctx.load(src),
                         "shots": int(rng.integers(1, 40)), "seed": 1000 + i})
    return reqs


def test_mixed_stream_completes_and_matches_alone_and_oracle(ctx):
    from paper_2604_11599_amd.serve import replay
    reqs = _trace(ctx)
    out = replay(ctx, reqs, hbm_budget=64 << 20, shots_per_tick=16)
    assert out["completed"] == len(reqs) and out["unfinished"] == 0
    for r in reqs[:12]:
        alone = replay(ctx, [dict(r, arrival=0.0)], hbm_budget=64 << 20, shots_per_tick=16)
        a, b = out["results"][r["id"]], alone["results"][r["id"]]
        if r["kind"] == "vqe":
            assert a[0] == b[0] and np.array_equal(a[1], b[1])
            e, g = r["prog"].expval_grad(r["theta"][None, :], r["coeffs"], r["codes"])
            assert abs(e[0] - a[0]) < 1e-12 and np.max(np.abs(g[0] - a[1])) < 1e-12
        else:
            assert np.array_equal(a.creg, b.creg) and np.array_equal(a.record_prob, b.record_prob)
            bits = a.bits()
            for s in range(min(r["shots"], 4)):
                o = sim.run_shot(r["src"], seed=r["seed"], shot=s)
                if any(abs(e[3] - e[4]) < 1e-12 for e in o.events):
                    continue
                assert list(bits[s]) == o.cbits
                assert abs(a.record_prob[s] - o.record_prob) < 1e-12


def test_tight_budget_admits_one_at_a_time(ctx):
    from paper_2604_11599_amd.serve import replay
    reqs = [r for r in _trace(ctx, count=12, seed=9) if r["kind"] == "shots"]
    loose = replay(ctx, reqs, hbm_budget=1 << 30, shots_per_tick=8)
    tight = replay(ctx, reqs, hbm_budget=1, shots_per_tick=8)
    for r in reqs:
        a, b = loose["results"][r["id"]], tight["results"][r["id"]]
        assert np.array_equal(a.creg, b.creg) and np.array_equal(a.record_prob, b.record_prob)


def test_expval_grad_each_equals_separate_calls_and_oracle(ctx):
    """One sweep over vectors with their own Hamiltonians (what the serving
    engine's energy lane batches) equals one call per vector bit for bit, and
    the oracle's adjoint."""
    src = W.c4_ansatz(8, 2)
    prog = ctx.load(src)
    hams = [W.c4_hamiltonian(seed=50 + k, n=8, terms=6 + k) for k in range(5)]
    th = W.c4_thetas(seed=3, batch=5, n_params=32)
    e, g = prog.expval_grad_each(th, hams)
    for k in range(5):
        e1, g1 = prog.expval_grad(th[k:k + 1], *hams[k])
        assert e[k] == e1[0] and np.array_equal(g[k], g1[0])
        eo, go = sim.grad_adjoint(src, th[k], *hams[k])
        assert abs(e[k] - eo) < 1e-12 and np.max(np.abs(g[k] - go)) < 1e-11


def test_lanes_overlap_and_late_arrivals_join(ctx):
    """Requests submitted while the lanes work (wide, persistent and energy at
    once) are admitted at the next step and finish with the results they have
    alone."""
    from paper_2604_11599_amd.serve import Server
    wide = ctx.load(W.c1_program(seed=5, n=21, layers=6, sites=(2, 4)))
    small = ctx.load(W.c1_program(seed=6, n=9, layers=5, sites=(1, 3)))
    vqe = ctx.load(W.c4_ansatz(8, 2))
    coeffs, codes = W.c4_hamiltonian(seed=9, n=8, terms=8)
    th = W.c4_thetas(seed=4, batch=1, n_params=32)[0]
    srv = Server(ctx, 1 << 34, shots_per_tick=16)
    try:
        t_w = srv.submit(wide, 12, seed=1)
        srv.step()
        t_s = srv.submit(small, 70, seed=2)      # arrives while the wide lane works
        t_v = srv.submit_expval_grad(vqe, th, coeffs, codes)
        done = {}
        while len(done) < 3:
            srv.step()
            for t in (t_w, t_s, t_v):
                if t not in done and srv.done(t):
                    done[t] = srv.fetch(t)
        a = wide.run_shots(12, seed=1, share=True)
        assert np.array_equal(done[t_w].creg, a.creg) and np.array_equal(done[t_w].record_prob, a.record_prob)
        b = ctx.run_batch([{"prog": small, "shots": 70, "seed": 2}])[0]
        assert np.array_equal(done[t_s].creg, b.creg) and np.array_equal(done[t_s].record_prob, b.record_prob)
        e, g = vqe.expval_grad(th[None, :], coeffs, codes)
        assert done[t_v][0] == e[0] and np.array_equal(done[t_v][1], g[0])
    finally:
        srv.close()
