"""GPU parity: libqsv (through its C ABI) against the CPU oracle.

Bars: forced-mode records and classical bits bit-exact; amplitudes within 1e-10
absolute; record (branch) probabilities within 1e-12; sampled shots equal to
the oracle's shot by shot except where a draw lies within 1e-12 of its
threshold; sampled histograms pass a chi-square test at p > 0.01.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sim

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-10
PROB_TOL = 1e-12
TIE = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_11599_amd import Context
    c = Context(0)
    yield c
    c.close()


def _bits_int(bits):
    return sum(int(b) << i for i, b in enumerate(bits))


def _near_tie(events, tie=TIE):
    return any(abs(e[3] - e[4]) < tie for e in events)


def _check_shots(ctx, src, n_shots, seed=11, theta=None, forced_from_oracle=False, state=True, noise=(0.0, 0.0),
                 share=False):
    say("case", src.splitlines()[2:4], "shots", n_shots, "seed", seed, "noise", noise)
    prog = ctx.load(src)
    oracle = [sim.run_shot(src, theta, seed=seed, shot=s, readout_error=noise[0], reset_error=noise[1])
              for s in range(n_shots)]
    forced = None
    if forced_from_oracle:
        width = max(1, max(len(o.record) for o in oracle))
        forced = np.zeros((n_shots, width), dtype=np.uint8)
        for s, o in enumerate(oracle):
            forced[s, :len(o.record)] = o.record
    res = prog.run_shots(n_shots, theta=theta, seed=seed, forced=forced, state_out=state, share=share,
                         readout_error=noise[0], reset_error=noise[1])
    bits = res.bits()
    skipped = 0
    for s, o in enumerate(oracle):
        if not forced_from_oracle and _near_tie(o.events):
            skipped += 1
            continue
        assert res.shot_status[s] == 0
        assert list(bits[s]) == o.cbits, f"shot {s}"
        assert list(res.record[s, :len(o.record)]) == o.record
        assert res.n_events[s] == o.words_drawn
        assert abs(res.record_prob[s] - o.record_prob) < PROB_TOL
    if state:
        assert np.max(np.abs(res.state - oracle[0].psi)) < AMP_TOL
    assert skipped <= n_shots // 10
    return res, oracle


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 12, 13, 14, 16])
def test_random_dynamic_programs_sampled(ctx, n):
    for seed in range(3):
        src = W.random_dynamic_program(1000 * n + seed, n, n_ops=60, final_measure=(seed == 2))
        _check_shots(ctx, src, 6, seed=seed)


@pytest.mark.parametrize("n", [4, 12, 15])
def test_random_dynamic_programs_forced(ctx, n):
    for seed in range(3):
        src = W.random_dynamic_program(77 * n + seed, n, n_ops=50, final_measure=True)
        _check_shots(ctx, src, 5, seed=seed + 40, forced_from_oracle=True)


def test_static_multi_tile_gates_on_every_qubit(ctx):
    rng = np.random.default_rng(5)
    for n in (13, 16, 18):
        lines = [W.circuits.HEADER, f"qubit[{n}] q;"]
        for _ in range(6 * n):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            t = [float(x) for x in rng.uniform(0, 6.283, 3)]
            lines += [f"U({t[0]!r}, {t[1]!r}, {t[2]!r}) q[{a}];", f"cx q[{a}], q[{b}];",
                      f"cp({t[0]!r}) q[{b}], q[{a}];", f"swap q[{b}], q[{(a + 1) % n if (a + 1) % n != b else a}];"]
        src = "\n".join(lines) + "\n"
        _check_shots(ctx, src, 1, state=True)


def test_c1_forced_records_and_sampled_shots(ctx):
    from scipy import stats
    src = W.c1_program(1)
    prog = ctx.load(src)
    total = 0.0
    probs = []
    for rec in range(8):
        forced = [(rec >> i) & 1 for i in range(3)]
        o = sim.run_shot(src, seed=3, shot=rec, forced=forced)
        r = prog.run_shots(1, seed=3, shot_offset=rec, forced=np.array([forced], np.uint8))
        assert list(r.bits()[0]) == o.cbits
        p_mid = np.prod([e[4] if e[2] == 0 else 1 - e[4] for e in o.events[:6]])
        probs.append(p_mid)
        assert abs(r.record_prob[0] - o.record_prob) < PROB_TOL
        total += p_mid
    assert abs(total - 1.0) < 1e-12
    # 1000 sampled shots: per-shot equality with the oracle, then chi-square of the mid-circuit records
    res, oracle = _check_shots(ctx, src, 1000, seed=21, state=False)
    obs = np.bincount([_bits_int(res.record[s, :3]) for s in range(1000)], minlength=8)
    exp = np.array(probs) * 1000
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < 1e-9:
        o, e = o[:-1], e[:-1]
    assert stats.chisquare(o, e).pvalue > 0.01


@pytest.mark.parametrize("prep", ["plus", "minus"])
def test_conditional_reset_10k_shots(ctx, prep):
    prog = ctx.load(W.conditional_reset_program(prep))
    r = prog.run_shots(10000, seed=7)
    b = r.bits()
    assert np.all(b[:, 1] == 0)
    assert 4700 < b[:, 0].sum() < 5300


def test_teleportation_and_if_else_states(ctx):
    src = W.teleport_program(0.4, 1.3, -2.1)
    prog = ctx.load(src)
    for rec in range(4):
        forced = np.array([[rec & 1, rec >> 1]], np.uint8)
        r = prog.run_shots(1, forced=forced, state_out=True)
        assert abs(r.record_prob[0] - 0.25) < PROB_TOL
        assert np.sum(np.abs(r.state.reshape(2, 4)[1]) ** 2) < 1e-24
        o = sim.run_shot(src, forced=list(forced[0]))
        assert np.max(np.abs(r.state - o.psi)) < AMP_TOL
    th = 1.234
    prog = ctx.load(W.if_else_program(th))
    for m in (0, 1):
        r = prog.run_shots(1, forced=np.array([[m]], np.uint8), state_out=True)
        psi = r.state.reshape(2, 2)
        expect = (np.array([math.cos(th / 2), -1j * math.sin(th / 2)]) if m
                  else np.array([np.exp(-0.5j * th), 0]))
        assert np.allclose(psi[:, m], expect, atol=1e-15)


def test_multibit_predicate_and_loops(ctx):
    for bits in range(16):
        src = W.multibit_predicate_program(bits)
        _check_shots(ctx, src, 1)
    _check_shots(ctx, W.rus_program(2.1, 8), 300, seed=4, state=False)
    _check_shots(ctx, W.c3_program(3, n=14, layers=4), 64, seed=9, state=False)


def test_rus_trip_count_distribution(ctx):
    from scipy import stats
    phi, K, shots = 2.1, 8, 20000
    s = math.cos(phi / 2) ** 2
    r = ctx.load(W.rus_program(phi, K)).run_shots(shots, seed=99)
    # a shot that stopped after T < K tries consumed 2T - 1 events (T measures, T - 1 resets);
    # one that ran out consumed 2K
    meas = (r.n_events.astype(np.int64) + 1) // 2
    expect = np.array([(1 - s) ** (k - 1) * s for k in range(1, K)] + [(1 - s) ** (K - 1)])
    obs = np.bincount(meas, minlength=K + 1)[1:]
    assert stats.chisquare(obs, expect * shots).pvalue > 0.01


def test_edge_cases(ctx):
    # empty program, zero shots, program starting with a measurement, forced zero probability
    r = ctx.load("qubit[3] q;").run_shots(2, state_out=True)
    assert abs(r.state[0] - 1) < 1e-15 and np.sum(np.abs(r.state[1:])) == 0
    assert ctx.load("qubit[2] q; bit c; c = measure q[0];").run_shots(0).creg.shape == (0, 1)
    _check_shots(ctx, "qubit[3] q; bit[2] c; c[0] = measure q[1]; h q[0]; c[1] = measure q[0];", 20)
    r = ctx.load("qubit[1] q; bit c; c = measure q[0]; x q[0];").run_shots(
        3, forced=np.array([[1], [0], [1]], np.uint8))
    assert list(r.shot_status) == [-6, 0, -6]
    from paper_2604_11599_amd import QsvError
    p = ctx.load("input float[64] t; qubit[1] q; rx(t) q[0];")
    with pytest.raises(ValueError):
        p.run_shots(1)
    with pytest.raises(QsvError):
        ctx.load(W.if_else_program(0.2)).expval(np.zeros((1, 0)), [1.0], [[3, 0]])


def test_determinism_and_batch_independence(ctx):
    src = W.c3_program(5, n=15, layers=3)
    prog = ctx.load(src)
    a = prog.run_shots(48, seed=1)
    b = prog.run_shots(48, seed=1)
    assert np.array_equal(a.creg, b.creg) and np.array_equal(a.record_prob, b.record_prob)
    for k in (0, 17, 47):
        one = prog.run_shots(1, seed=1, shot_offset=k)
        assert np.array_equal(one.creg[0], a.creg[k])
        assert one.record_prob[0] == a.record_prob[k]


def _same_results(a, b, state=True):
    assert np.array_equal(a.creg, b.creg) and np.array_equal(a.record, b.record)
    assert np.array_equal(a.record_prob, b.record_prob) and np.array_equal(a.n_events, b.n_events)
    assert np.array_equal(a.shot_status, b.shot_status)
    if state:
        assert np.array_equal(a.state, b.state)


def test_trajectory_sharing_is_bit_identical(ctx):
    """Shots with equal histories share one state; results equal running every
    shot on its own, bit for bit (mid-circuit multi-qubit measurement with
    feed-forward, resets, repeat-until-success loops, random dynamic programs,
    forced records, many shots)."""
    cases = [(W.c2_program(2, n=14, layers=8), 24), (W.c1_program(4), 40), (W.c3_program(6, n=13, layers=3), 200),
             (W.random_dynamic_program(3, 13, n_ops=60), 64), (W.random_dynamic_program(8, 14, n_ops=50), 33)]
    for src, shots in cases:
        say("trajectory sharing case", src.splitlines()[2:3], shots, "shots")
        prog = ctx.load(src)
        a = prog.run_shots(shots, seed=5, state_out=True)
        b = prog.run_shots(shots, seed=5, state_out=True, share=True)
        _same_results(a, b)
        c = prog.run_shots(shots, seed=9, shot_offset=7, share=True)
        d = prog.run_shots(shots, seed=9, shot_offset=7)
        _same_results(c, d, state=False)
    # forced records: every shot its own forced row
    src = W.c1_program(4)
    prog = ctx.load(src)
    forced = np.array([[(k >> j) & 1 for j in range(3)] for k in range(8)] * 3, dtype=np.uint8)
    _same_results(prog.run_shots(24, seed=1, forced=forced), prog.run_shots(24, seed=1, forced=forced, share=True),
                  state=False)


def test_trajectory_sharing_runs_passes_once_per_history():
    """The repeat-until-success loop of a 13-qubit circuit has at most 9
    histories before the final measure-all: with 256 shots the shared run moves
    at most 9/256 of the per-shot gate-pass bytes."""
    from paper_2604_11599_amd import Context
    c = Context(0, profile=True)
    try:
        prog = c.load(W.c3_program(6, n=13, layers=3))
        c.profile_reset()
        prog.run_shots(256, seed=3)
        full = c.profile()["pass_uncond_bytes"]
        c.profile_reset()
        prog.run_shots(256, seed=3, share=True)
        shared = c.profile()["pass_uncond_bytes"]
        assert 0 < shared <= full * 9 / 256
    finally:
        c.close()


def test_gate_modifiers_match_oracle(ctx):
    """inv @, pow(k) @, ctrl @, negctrl @ programs (lowered to standard gates)
    against the oracle, which applies the modifiers by definition."""
    for seed, n in [(0, 6), (1, 11), (2, 13)]:
        _check_shots(ctx, W.modifier_program(seed, n, 60), 24, seed=seed)


def test_logical_conditions_match_oracle(ctx):
    """if conditions with &&, || and ! (disjoint flag guards) on the tile path,
    with and without trajectory sharing, and in a persistent batch."""
    for seed, n in [(1, 4), (2, 9), (3, 13), (4, 16)]:
        src = W.logic_program(seed, n, n_ops=40)
        _check_shots(ctx, src, 8, seed=seed, state=n <= 13)
        _check_shots(ctx, src, 8, seed=seed + 10, forced_from_oracle=True, state=False)
        _check_shots(ctx, src, 8, seed=seed, state=False, share=True)
        o = sim.run_shots(src, 8, seed=7)
        r = ctx.run_batch([{"prog": ctx.load(src), "shots": 8, "seed": 7}])[0]
        for s in range(8):
            if _near_tie(sim.run_shot(src, seed=7, shot=s).events):
                continue
            assert list(r.record[s, :len(o[s]["record"])]) == o[s]["record"]


def test_run_option_validation_and_complex64_with_noise(ctx):
    """Error rates outside [0, 1) are rejected before any work; readout and
    reset errors in complex64 draw the same words as in complex128, so the
    records agree shot by shot with the noisy oracle outside the tie band."""
    from paper_2604_11599_amd import QsvError
    prog = ctx.load(W.c1_program(4))
    for kw in ({"readout_error": 1.0}, {"reset_error": -0.1}, {"readout_error": float("nan")}):
        with pytest.raises(QsvError):
            prog.run_shots(4, seed=1, **kw)
    src = W.random_dynamic_program(41, 13, n_ops=60)
    noise = (0.05, 0.08)
    res = ctx.load(src).run_shots(16, seed=2, complex64=True, readout_error=noise[0], reset_error=noise[1])
    checked = 0
    for s in range(16):
        o = sim.run_shot(src, seed=2, shot=s, readout_error=noise[0], reset_error=noise[1])
        if _near_tie(o.events, C64_TIE):
            continue
        assert list(res.record[s, :len(o.record)]) == o.record and res.n_events[s] == o.words_drawn
        checked += 1
    assert checked >= 12


def test_multi_controlled_gates_match_oracle(ctx):
    """ctrl(k) @ and controls on two-qubit gates (lowered through CX
    decompositions and Toffolis) on a 13-qubit dynamic program: shots and the
    final state against the oracle's by-definition matrices."""
    body = ("ctrl(2) @ x q[0], q[5], q[12]; ctrl @ swap q[3], q[7], q[11]; negctrl @ ctrl @ h q[1], q[2], q[9];"
            "ctrl(2) @ U(0.4, 1.2, -0.7) q[4], q[8], q[10]; ctrl @ crx(0.9) q[6], q[0], q[3];")
    head = W.random_dynamic_program(77, 13, n_ops=40, final_measure=True)
    assert head.endswith("f = measure q;\n")
    src = head[:-len("f = measure q;\n")] + body.replace(";", ";\n") + "f = measure q;\n"
    _check_shots(ctx, src, 8, seed=3)
    _check_shots(ctx, src, 8, seed=4, forced_from_oracle=True, state=False)


def test_classical_assignment_matches_oracle(ctx):
    """c[i] = <condition> and c = <integer> (set / clear bit events) on the tile
    path, with and without trajectory sharing, and in a persistent batch."""
    for seed, n in [(11, 4), (12, 13)]:
        src = W.logic_program(seed, n, n_ops=40, assign=True)
        _check_shots(ctx, src, 8, seed=seed, state=n <= 13)
        _check_shots(ctx, src, 8, seed=seed + 10, forced_from_oracle=True, state=False)
        _check_shots(ctx, src, 8, seed=seed, state=False, share=True)
        o = sim.run_shots(src, 8, seed=7)
        r = ctx.run_batch([{"prog": ctx.load(src), "shots": 8, "seed": 7}])[0]
        bits = r.bits()
        for s in range(8):
            if _near_tie(sim.run_shot(src, seed=7, shot=s).events):
                continue
            assert list(r.record[s, :len(o[s]["record"])]) == o[s]["record"]
            assert list(bits[s]) == sim.run_shot(src, seed=7, shot=s).cbits


def test_readout_and_reset_errors_match_oracle(ctx):
    """Readout and reset errors drawn from each shot's own Philox stream: shot by
    shot equal to the oracle on the tile-pass path (with and without trajectory
    sharing) and in a persistent batch; the noisy conditional reset's flip rate
    is the closed form 2 e (1 - e)."""
    noise = (0.07, 0.05)
    for src, shots in [(W.c1_program(4), 64), (W.random_dynamic_program(31, 13, n_ops=60), 32),
                       (W.c3_program(6, n=13, layers=3), 32)]:
        _check_shots(ctx, src, shots, seed=3, noise=noise, state=False)
        _check_shots(ctx, src, shots, seed=3, noise=noise, state=False, share=True)
        o = sim.run_shots(src, shots, seed=5, readout_error=noise[0], reset_error=noise[1])
        r = ctx.run_batch([{"prog": ctx.load(src), "shots": shots, "seed": 5, "readout_error": noise[0],
                            "reset_error": noise[1]}])[0]
        for s in range(shots):
            if _near_tie(sim.run_shot(src, seed=5, shot=s, readout_error=noise[0], reset_error=noise[1]).events):
                continue
            assert list(r.record[s, :len(o[s]["record"])]) == o[s]["record"] and r.n_events[s] == o[s]["n_events"]
    e = 0.1
    src = W.circuits.HEADER + "qubit[1] q;\nbit c;\nbit f;\nh q[0];\nc = measure q[0];\nif (c == 1) x q[0];\nf = measure q[0];\n"
    res = ctx.load(src).run_shots(20000, seed=9, readout_error=e)
    frac = float(np.mean((res.creg[:, 0] >> 1) & 1))
    p = 2 * e * (1 - e)
    assert abs(frac - p) < 4 * math.sqrt(p * (1 - p) / 20000)


# ---------------------------------------------------------------------------
# complex64 state (single-precision amplitudes and matrix-core products)
#
# Unit roundoff 2^-24 = 6e-8. A dense phase is a 16-term complex product, so it
# adds at most about 20 roundoffs to the state's 2-norm error (1.2e-6); the
# programs below have at most ~15 phases and gate lists per shot, so the state
# error stays below 2e-5 in the 2-norm, the bound the amplitude check uses.
# Probabilities are sums of squares of those amplitudes (relative error below
# 4e-5), so outcomes are compared shot by shot except where the oracle's draw
# lies within 1e-4 of its threshold (the decision is not fixed there at
# single precision); forced records are compared bit for bit.
# ---------------------------------------------------------------------------
C64_AMP = 2e-5
C64_PROB = 4e-5
C64_TIE = 1e-4


def _check_c64(ctx, src, n_shots, seed=11, forced_from_oracle=False, share=False, state=True):
    say("c64 case", src.splitlines()[2:4], "shots", n_shots, "seed", seed, "forced", forced_from_oracle, "share", share)
    prog = ctx.load(src)
    oracle = [sim.run_shot(src, seed=seed, shot=s) for s in range(n_shots)]
    forced = None
    if forced_from_oracle:
        width = max(1, max(len(o.record) for o in oracle))
        forced = np.zeros((n_shots, width), dtype=np.uint8)
        for s, o in enumerate(oracle):
            forced[s, :len(o.record)] = o.record
    res = prog.run_shots(n_shots, seed=seed, forced=forced, state_out=state, share=share, complex64=True)
    bits = res.bits()
    skipped = 0
    for s, o in enumerate(oracle):
        if not forced_from_oracle and _near_tie(o.events, C64_TIE):
            skipped += 1
            continue
        assert res.shot_status[s] == 0
        assert list(bits[s]) == o.cbits, f"shot {s}"
        assert list(res.record[s, :len(o.record)]) == o.record
        assert res.n_events[s] == o.words_drawn
        assert abs(res.record_prob[s] - o.record_prob) <= C64_PROB * o.record_prob
    if state and (forced_from_oracle or not _near_tie(oracle[0].events, C64_TIE)):
        err = float(np.linalg.norm(res.state - oracle[0].psi))
        say("  c64 state error (2-norm)", err)
        assert err < C64_AMP
    assert skipped <= n_shots // 5
    return res


@pytest.mark.parametrize("n", [2, 3, 8, 12, 13, 16])
def test_complex64_random_dynamic_programs(ctx, n):
    for seed in range(2):
        src = W.random_dynamic_program(500 * n + seed, n, n_ops=60, final_measure=(seed == 1))
        _check_c64(ctx, src, 8, seed=seed)
        _check_c64(ctx, src, 8, seed=seed + 20, forced_from_oracle=True)
        _check_c64(ctx, src, 8, seed=seed, share=True, state=False)


def test_complex64_dense_passes_and_conditional_reset(ctx):
    """All-dense 12-bit passes (the eight-wave matrix-core pass) on a layered
    circuit with a mid-circuit measurement, and the conditional reset."""
    src = W.c2_program(n=14, layers=6, final_measure=False)
    _check_c64(ctx, src, 8, seed=4)
    _check_c64(ctx, src, 8, seed=4, forced_from_oracle=True)
    _check_c64(ctx, src, 16, seed=4, share=True, state=False)
    b = ctx.load(W.conditional_reset_program("plus")).run_shots(10000, seed=8, complex64=True).bits()
    assert np.all(b[:, 1] == 0) and 4700 < b[:, 0].sum() < 5300


def test_complex64_matches_complex128_at_20_qubits(ctx):
    """The same shots in both precisions: records equal, trajectory
    probabilities and final states within the single-precision bound."""
    src = W.c2_program(n=20, layers=12, final_measure=False)
    prog = ctx.load(src)
    r64 = prog.run_shots(4, seed=6, state_out=True, complex64=True)
    r128 = prog.run_shots(4, seed=6, state_out=True)
    assert np.array_equal(r64.record, r128.record) and np.array_equal(r64.creg, r128.creg)
    assert np.all(np.abs(r64.record_prob - r128.record_prob) <= C64_PROB * r128.record_prob)
    err = float(np.linalg.norm(r64.state - r128.state))
    say("  c64 vs c128 state error (2-norm), 20 qubits", err)
    assert err < C64_AMP
    assert abs(np.linalg.norm(r64.state) - 1.0) < C64_AMP


# ---------------------------------------------------------------------------
# Expectation values and gradients
# ---------------------------------------------------------------------------
def test_expval_and_gradient_small(ctx):
    n, layers = 6, 3
    src = W.c4_ansatz(n, layers)
    coeffs, codes = W.c4_hamiltonian(seed=3, n=n, terms=12)
    thetas = W.c4_thetas(seed=5, batch=5, n_params=2 * n * layers)
    prog = ctx.load(src)
    e = prog.expval(thetas, coeffs, codes)
    e2, g = prog.expval_grad(thetas, coeffs, codes)
    for b in range(5):
        eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
        assert abs(e[b] - eo) < 1e-12 and abs(e2[b] - eo) < 1e-12
        assert np.max(np.abs(g[b] - go)) < 1e-11
    gp = sim.grad_param_shift(src, thetas[0], coeffs, codes)
    assert np.max(np.abs(g[0] - gp)) < 1e-11


def test_gradient_matrix_core_sweep(ctx):
    """Passes of 2^10..2^12-amplitude tiles whose phases are all dense take the
    adjoint sweep on the matrix cores (tiles of 10, 11 and 12 bits, one to five
    passes, U and controlled rotations and phases inside the dense phases)."""
    from paper_2604_11599_amd import lower
    from paper_2604_11599_amd.api import plan_inspect
    cases = [(W.c4_ansatz(10, 2), 10, 40), (W.c4_ansatz(12, 3), 12, 72), (W.c4_ansatz(14, 4), 14, 112),
             (W.param_program(5, 11, 70, 24), 11, 24), (W.param_program(7, 13, 120, 40), 13, 40),
             (W.param_program(9, 14, 160, 50), 14, 50)]
    for src, n, P in cases:
        st = plan_inspect(lower(src), 0)
        assert st.n_mfma_sweep_passes == st.n_passes > 0
        coeffs, codes = W.c4_hamiltonian(seed=n, n=n, terms=16)
        thetas = W.c4_thetas(seed=100 + n, batch=3, n_params=P)
        say("matrix-core sweep case", n, "qubits", P, "params", st.n_passes, "passes")
        e, g = ctx.load(src).expval_grad(thetas, coeffs, codes)
        for b in range(3):
            eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
            assert abs(e[b] - eo) < 1e-12
            assert np.max(np.abs(g[b] - go)) < 1e-11


def test_gradient_through_gate_modifiers(ctx):
    """Parameters under inv @ and ctrl @ on a 12-qubit program (all-dense passes,
    matrix-core sweep) against the oracle's adjoint, which differentiates the
    modified matrices by definition."""
    n, P = 12, 24
    lines = ['OPENQASM 3.0;', 'include "stdgates.inc";', f"input array[float[64], {P}] t;", f"qubit[{n}] q;"]
    for k in range(P):
        a, b = k % n, (5 * k + 3) % n
        lines.append(f"h q[{a}];")
        lines.append([f"inv @ ry(t[{k}]) q[{a}];", f"ctrl @ rz(t[{k}]) q[{a}], q[{b}];",
                      f"ctrl @ U(t[{k}], 0.3, -0.2) q[{b}], q[{a}];", f"negctrl @ rx(2 * t[{k}]) q[{a}], q[{b}];"][k % 4])
        lines.append(f"cx q[{a}], q[{(a + 1) % n}];")
    src = "\n".join(lines) + "\n"
    from paper_2604_11599_amd import lower
    from paper_2604_11599_amd.api import plan_inspect
    st = plan_inspect(lower(src), 0)
    assert st.n_mfma_sweep_passes == st.n_passes > 0
    coeffs, codes = W.c4_hamiltonian(seed=21, n=n, terms=16)
    thetas = W.c4_thetas(seed=22, batch=2, n_params=P)
    e, g = ctx.load(src).expval_grad(thetas, coeffs, codes)
    for b in range(2):
        eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
        assert abs(e[b] - eo) < 1e-12
        assert np.max(np.abs(g[b] - go)) < 1e-11


def test_gradient_through_multi_controlled_gates(ctx):
    """Parameters under several controls and controls on two-qubit gates (the
    angle enters the decomposition as +-t/2 in several gates) against the
    oracle's adjoint of the controlled matrices, on 8 and 12 qubits."""
    for n, P in ((8, 12), (12, 16)):
        lines = ['OPENQASM 3.0;', 'include "stdgates.inc";', f"input array[float[64], {P}] t;", f"qubit[{n}] q;"]
        for k in range(P):
            a, b, c = k % n, (3 * k + 1) % n, (5 * k + 2) % n
            if len({a, b, c}) < 3:
                c = (max(a, b) + 1) % n
                if c in (a, b):
                    c = (c + 1) % n
            lines.append(f"h q[{a}];")
            lines.append([f"ctrl(2) @ ry(t[{k}]) q[{a}], q[{b}], q[{c}];", f"ctrl @ crz(t[{k}]) q[{c}], q[{a}], q[{b}];",
                          f"negctrl @ ctrl @ rx(2 * t[{k}]) q[{b}], q[{c}], q[{a}];",
                          f"ctrl @ cp(t[{k}] + 0.5) q[{a}], q[{c}], q[{b}];"][k % 4])
            lines.append(f"cx q[{a}], q[{(a + 1) % n}];")
        src = "\n".join(lines) + "\n"
        coeffs, codes = W.c4_hamiltonian(seed=31, n=n, terms=10)
        thetas = W.c4_thetas(seed=32, batch=2, n_params=P)
        e, g = ctx.load(src).expval_grad(thetas, coeffs, codes)
        for b in range(2):
            eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
            assert abs(e[b] - eo) < 1e-12
            assert np.max(np.abs(g[b] - go)) < 1e-11


def test_expval_closed_form_and_general_gates(ctx):
    prog = ctx.load(W.hea2_program())
    ab = np.array([[0.3, 1.1], [2.0, -0.4]])
    e, g = prog.expval_grad(ab, [1.0], [[3, 3]])
    assert np.allclose(e, np.cos(ab[:, 1]), atol=1e-14)
    assert np.allclose(g, np.stack([np.zeros(2), -np.sin(ab[:, 1])], 1), atol=1e-14)
    src = ('input array[float[64], 4] t; qubit[3] q; U(t[0], 2 * t[1], -t[2]) q[0]; cx q[0], q[1];'
           'crz(t[3]) q[1], q[2]; cp(t[1] + 0.3) q[2], q[0]; rx(t[2]) q[2]; h q[1]; cry(0.5 * t[0]) q[0], q[2];'
           'u2(t[3], t[0]) q[1]; swap q[0], q[2]; crx(t[1]) q[2], q[1]; p(t[2]) q[0]; ry(t[3]) q[1];')
    coeffs, codes = W.c4_hamiltonian(seed=8, n=3, terms=7)
    th = np.array([[0.7, -1.2, 2.5, 0.4], [1.9, 0.3, -0.8, -2.2]])
    e, g = ctx.load(src).expval_grad(th, coeffs, codes)
    for b in range(2):
        eo, go = sim.grad_adjoint(src, th[b], coeffs, codes)
        assert abs(e[b] - eo) < 1e-12 and np.max(np.abs(g[b] - go)) < 1e-11


def test_hamiltonian_tiles_local_and_remote_groups(ctx):
    """The H psi sweep on states larger than one amplitude tile: terms whose X
    masks lie inside the tile (partners read from LDS) and outside it (partners
    read from memory), several terms per X mask, Y counts of 0..3, an identity
    term and a term with X on every qubit, at 13 and 16 qubits, against the
    oracle's energy and adjoint gradient; per-vector Hamiltonians equal one call
    per vector bit for bit."""
    for n in (13, 16):
        src = W.c4_ansatz(n, 2)
        rng = np.random.default_rng(600 + n)
        base = rng.integers(0, 4, size=(24, n)).astype(np.uint8)
        same_x = base[:8].copy()                     # same X masks as the first 8, other Z parts
        flip = (same_x == 3) | (same_x == 0)
        same_x[flip] = 3 - same_x[flip]
        ys = np.zeros((4, n), dtype=np.uint8)
        for k in range(4):
            ys[k, rng.choice(n, size=k + 1, replace=False)] = 2
        codes = np.concatenate([base, same_x, ys, np.zeros((1, n), np.uint8), np.ones((1, n), np.uint8)])
        coeffs = rng.standard_normal(len(codes))
        thetas = W.c4_thetas(seed=700 + n, batch=2, n_params=4 * n)
        prog = ctx.load(src)
        say("hamiltonian tiles case", n, "qubits", len(codes), "terms")
        e, g = prog.expval_grad(thetas, coeffs, codes)
        for b in range(2):
            eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
            assert abs(e[b] - eo) < 1e-12
            assert np.max(np.abs(g[b] - go)) < 1e-11
        hams = [(coeffs, codes), W.c4_hamiltonian(seed=n, n=n, terms=20)]
        ee, ge = prog.expval_grad_each(thetas, hams)
        for b in range(2):
            e1, g1 = prog.expval_grad(thetas[b:b + 1], *hams[b])
            assert ee[b] == e1[0] and np.array_equal(ge[b], g1[0])


def test_c4_full_size_energy_and_fd(ctx):
    src = W.c4_ansatz(20, 6)
    coeffs, codes = W.c4_hamiltonian(seed=4, n=20, terms=60)
    thetas = W.c4_thetas(seed=44, batch=64, n_params=240)
    prog = ctx.load(src)
    e, g = prog.expval_grad(thetas, coeffs, codes)
    say("c4 oracle energy of vector 0")
    eo = sim.expval(src, thetas[0], coeffs, codes)
    assert abs(e[0] - eo) < 1e-10
    e_only = prog.expval(thetas, coeffs, codes)
    assert np.max(np.abs(e_only - e)) < 1e-12
    h = 1e-5
    for k in (0, 57, 239):
        tp, tm = thetas[:2].copy(), thetas[:2].copy()
        tp[:, k] += h
        tm[:, k] -= h
        fd = (prog.expval(tp, coeffs, codes) - prog.expval(tm, coeffs, codes)) / (2 * h)
        assert np.max(np.abs(fd - g[:2, k])) < 1e-7


def test_c4_full_size_gradient_matches_oracle_adjoint(ctx):
    """One full 240-entry gradient of the 20-qubit ansatz (the matrix-core
    sweep over every pass at the benchmark's size) against the oracle's plain
    adjoint sequence, and its energy, to 1e-10."""
    src = W.c4_ansatz(20, 6)
    coeffs, codes = W.c4_hamiltonian(seed=4, n=20, terms=60)
    thetas = W.c4_thetas(seed=44, batch=64, n_params=240)
    e, g = ctx.load(src).expval_grad(thetas, coeffs, codes)
    for b in (0, 63):
        say(f"c4 oracle adjoint of vector {b} (240 parameters, 20 qubits)")
        eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
        assert abs(e[b] - eo) < 1e-10
        err = float(np.max(np.abs(g[b] - go)))
        say("  max gradient error", err)
        assert err < 1e-10


# ---------------------------------------------------------------------------
# The headline workload's program (28-qubit brickwork with the 4-qubit site,
# the 0b1010 block and the if/else) at widths and depths the oracle runs in
# test time, in complex128.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,layers,sampled,records", [(14, 40, 12, range(16)), (20, 12, 3, (0b0101, 0b1010))])
def test_c2_program_complex128_matches_oracle(ctx, n, layers, sampled, records):
    """Sampled shots (with the final measure-all) shot by shot; forced records
    (c[0..3]; at 14 qubits all 16) bit-exact with their probabilities and the
    state before the measure-all within 1e-10 per amplitude."""
    full = W.c2_program(seed=2, n=n, layers=layers, final_measure=True)
    _check_shots(ctx, full, sampled, seed=5, state=False)
    nomeas = W.c2_program(seed=2, n=n, layers=layers, final_measure=False)
    prog = ctx.load(nomeas)
    taken = 0
    for rec in records:
        forced = [(rec >> i) & 1 for i in range(4)]
        o = sim.run_shot(nomeas, seed=9, shot=rec, forced=forced)
        r = prog.run_shots(1, seed=9, shot_offset=rec, forced=np.array([forced], np.uint8), state_out=True)
        assert r.shot_status[0] == o.status
        if o.status:
            continue
        taken += 1
        assert list(r.bits()[0]) == o.cbits
        assert list(r.record[0]) == o.record
        assert abs(r.record_prob[0] - o.record_prob) < PROB_TOL
        assert np.max(np.abs(r.state - o.psi)) < AMP_TOL
    assert taken >= 2


# ---------------------------------------------------------------------------
# Classical integer expressions and variables on the device (expression code
# evaluated by the event interpreter: CSTORE and expression predicates)
# ---------------------------------------------------------------------------
CLASSICAL_BODIES = [
    "d = c + 1; t = c > d; int[8] x = c * 3 - d; uint[5] u = (c << 2) | d; x >>= 1; u ^= x; "
    "if (u > x) rx(0.7) q[5]; t = measure q[5];",
    "if (c == d) x q[3]; if (c < d && (c & 1) == 0) h q[3]; if (!(c + d > 4) || c ^ d) x q[3]; t = measure q[3];",
    "uint[4] n = 0; for uint i in [0:2] { h q[i + 6]; d[i] = measure q[i + 6]; if (d[i]) n += 1; } "
    "if (n >= 2) x q[3]; t = measure q[3]; c = n;",
    "int[6] y = -5; y = y / 2 + c % 3; int[16] z = (y << 3) >> 1; uint[3] w = z; if (y < 0) x q[4]; "
    "t = measure q[4];",
]


def _classical_src(body, n=14, seed=0):
    rng = np.random.default_rng(seed)
    lines = [W.circuits.HEADER, f"qubit[{n}] q;", "bit[3] c;", "bit[3] d;", "bit t;"]
    for q in range(n):
        t = [float(x) for x in rng.uniform(0, 6.283, 3)]
        lines.append(f"U({t[0]!r}, {t[1]!r}, {t[2]!r}) q[{q}];")
    for q in range(0, n - 1, 2):
        lines.append(f"cx q[{q}], q[{q + 1}];")
    lines += ["c[0] = measure q[0];", "c[1] = measure q[1];", "c[2] = measure q[2];", "d = c;", body]
    for q in range(n):
        lines.append(f"ry({0.3 + 0.1 * q!r}) q[{q}];")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("k", range(len(CLASSICAL_BODIES)))
def test_classical_expressions_match_oracle(ctx, k):
    src = _classical_src(CLASSICAL_BODIES[k], seed=k)
    _check_shots(ctx, src, 10, seed=30 + k)
    _check_shots(ctx, src, 10, seed=40 + k, share=True, state=False)
    _check_shots(ctx, src, 6, seed=50 + k, forced_from_oracle=True)
    # the persistent interpreter (12 qubits in LDS, 13 in an HBM slot)
    for n in (12, 13):
        s2 = _classical_src(CLASSICAL_BODIES[k], n=n, seed=k)
        res = ctx.run_batch([{"prog": ctx.load(s2), "shots": 12, "seed": 7}])[0]
        bits = res.bits()
        for s in range(12):
            o = sim.run_shot(s2, seed=7, shot=s)
            if _near_tie(o.events):
                continue
            assert list(bits[s]) == o.cbits
            assert abs(res.record_prob[s] - o.record_prob) < PROB_TOL


# ---------------------------------------------------------------------------
# Gate angles that combine several inputs (derived parameters formed on the
# device before binding; gradients reach every input through the chain rule)
# ---------------------------------------------------------------------------
def _multi_input_program(n, measure):
    lines = [W.circuits.HEADER, "input array[float[64], 4] t;", "input float[64] s;", f"qubit[{n}] q;"]
    if measure:
        lines.append(f"bit[{n}] c;")
    for layer in range(3):
        for q in range(n):
            lines.append([f"rx(t[0] + t[1] * {q + 1}) q[{q}];", f"ry(2 * t[2] - t[{q % 4}] + 0.3) q[{q}];",
                          f"U(t[3] - s, t[1] + t[2], s / 2 + t[{(q + layer) % 4}]) q[{q}];"][(q + layer) % 3])
        for q in range(layer % 2, n - 1, 2):
            lines.append(f"crz(t[0] + s) q[{q}], q[{q + 1}];" if q % 4 == 0 else f"cx q[{q}], q[{q + 1}];")
    if measure:
        lines.append("c = measure q;")
    return "\n".join(lines) + "\n"


def test_angles_combining_inputs_shots_and_gradients(ctx):
    th = np.array([0.4, -1.1, 2.3, 0.7, -0.35])
    dyn = _multi_input_program(13, True)
    _check_shots(ctx, dyn, 6, seed=3, theta=th, state=False)
    res = ctx.run_batch([{"prog": ctx.load(dyn), "shots": 6, "seed": 3, "theta": th}])[0]
    for s in range(6):
        o = sim.run_shot(dyn, th, seed=3, shot=s)
        if not _near_tie(o.events):
            assert list(res.bits()[s]) == o.cbits
    src = _multi_input_program(12, False)
    coeffs, codes = W.c4_hamiltonian(seed=12, n=12, terms=14)
    thetas = np.stack([th, th[::-1] * 0.7, th + 1.0])
    prog = ctx.load(src)
    e, g = prog.expval_grad(thetas, coeffs, codes)
    for b in range(3):
        eo, go = sim.grad_adjoint(src, thetas[b], coeffs, codes)
        assert abs(e[b] - eo) < 1e-12 and np.max(np.abs(g[b] - go)) < 1e-11
    h = 1e-5
    for k in range(5):
        tp, tm = thetas[:1].copy(), thetas[:1].copy()
        tp[0, k] += h
        tm[0, k] -= h
        fd = (prog.expval(tp, coeffs, codes)[0] - prog.expval(tm, coeffs, codes)[0]) / (2 * h)
        assert abs(fd - g[0, k]) < 1e-7
