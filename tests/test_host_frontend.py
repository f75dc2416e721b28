"""CPU tests of the product's host side: ABI surface, lowering and planning."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2604_11599_amd import QasmError, lower
from paper_2604_11599_amd import _abi
from tests import ir_interp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------------------
# ABI surface
# ---------------------------------------------------------------------------
def _declared_functions():
    names = set()
    for h in ("qsv.h", "qsv_plan.h", "qsv_diag.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(qsv_[a-z_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    declared = _declared_functions()
    assert {"qsv_create", "qsv_load_program", "qsv_run_shots", "qsv_expval", "qsv_expval_grad"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(_abi.SIGNATURES) == declared


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without libqsv.so the binding raises instead of falling back to anything
    else (there is no CPU path in the product)."""
    from paper_2604_11599_amd import _abi
    with pytest.raises(ImportError):
        _abi.load_library(str(tmp_path / "libqsv.so"))
    monkeypatch.setattr(_abi, "_LIB", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "libqsv.so"))
    monkeypatch.setattr(_abi.load_library, "__defaults__", (str(tmp_path / "libqsv.so"),))
    with pytest.raises(ImportError):
        _abi.lib()


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures and numpy record types against the C
    compiler's own sizeof/offsetof of include/qsv.h."""
    import shutil
    import subprocess
    from paper_2604_11599_amd.lower import COP_DTYPE, INSTR_DTYPE, LIN_DTYPE, NOISE_DTYPE, PRED_DTYPE
    checks = {"qsv_config": _abi.Config, "qsv_program_desc": _abi.ProgramDesc, "qsv_run_opts": _abi.RunOpts,
              "qsv_shot_results": _abi.ShotResults, "qsv_pauli_sum": _abi.PauliSum, "qsv_request": _abi.Request,
              "qsv_profile": _abi.Profile, "qsv_plan_options": _abi.PlanOptions, "qsv_tune_report": _abi.TuneReport,
              "qsv_program_info": _abi.ProgramInfo, "qsv_plan_stats": _abi.PlanStats}
    dtypes = {"qsv_instr": INSTR_DTYPE, "qsv_pred": PRED_DTYPE, "qsv_cop": COP_DTYPE, "qsv_lin": LIN_DTYPE,
              "qsv_noise": NOISE_DTYPE}
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qsv.h"', '#include "qsv_plan.h"',
             'int main(void) {']
    for name, st in checks.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    for name, dt in dtypes.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in dt.names:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    (tmp_path / "probe.c").write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(tmp_path / "probe.c"), "-o",
                    str(tmp_path / "probe")], check=True)
    out = dict(line.split() for line in subprocess.run([str(tmp_path / "probe")], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for name, st in checks.items():
        assert ctypes.sizeof(st) == int(out[name]), name
        for f, _ in st._fields_:
            assert getattr(st, f).offset == int(out[f"{name}.{f}"]), (name, f)
    for name, dt in dtypes.items():
        assert dt.itemsize == int(out[name]), name
        for f in dt.names:
            assert dt.fields[f][1] == int(out[f"{name}.{f}"]), (name, f)


# ---------------------------------------------------------------------------
# Lowering == oracle (through a test-only interpreter of the instruction stream)
# ---------------------------------------------------------------------------
def _compare(src, theta=(), shots=3, seed=5, forced=None):
    lp = lower(src)
    for shot in range(shots):
        o = sim.run_shot(src, theta if len(theta) else None, seed=seed, shot=shot, forced=forced)
        psi, bits, record = ir_interp.run(lp, theta, seed=seed, shot=shot, forced=forced)
        assert bits == o.cbits and record == o.record
        assert np.max(np.abs(psi - o.psi)) < 1e-13


@pytest.mark.parametrize("seed", range(20))
def test_lowering_matches_oracle_random_dynamic(seed):
    _compare(W.random_dynamic_program(seed, 2 + seed % 5, n_ops=40, final_measure=seed % 2 == 0))


def test_lowering_protocols():
    _compare(W.conditional_reset_program("plus"), shots=6)
    _compare(W.teleport_program(0.3, 1.2, -0.7), shots=6)
    _compare(W.if_else_program(0.77), shots=4)
    for b in (0, 10, 5):
        _compare(W.multibit_predicate_program(b), shots=1)
    _compare(W.rus_program(2.0, 5), shots=8)
    _compare(W.c1_program(1), shots=2)
    _compare(W.c3_program(3, n=6, layers=2, max_iter=4), shots=5)
    _compare(W.qft_program(4, 5), shots=1)


def test_lowering_parameters_and_custom_gates():
    src = ('OPENQASM 3.0; input array[float[64], 3] th; input float[64] s; qubit[3] q; bit[2] c;'
           'const float[64] k = pi / 3;'
           'gate rot(a, b) x, y { ry(a) x; cx x, y; rz(b - k) y; } '
           'rot(2 * th[0] + 0.25, th[1] / 4) q[0], q[2]; u2(s, -th[2]) q[1]; U(th[0], s, k) q[2];'
           'c[0] = measure q[0]; if (c[0] == 1) { crx(s * 3) q[1], q[2]; } else cp(th[1]) q[2], q[0];')
    _compare(src, theta=np.array([0.3, -1.1, 2.2, 0.9]), shots=4)


def test_nested_loops_break_continue():
    src = ('qubit[3] q; bit[3] c;'
           'for uint i in [0:2] { h q[i]; c[i] = measure q[i]; if (c[i] == 1) continue; '
           '  for uint j in [1:2] { rx(0.3 * j) q[(i + j) % 3]; if (c[0]) break; } x q[i]; }'
           'for int k in [2:-1:0] { ry(0.1 * k) q[k]; }')
    _compare(src, shots=8)


def test_lowering_errors():
    for bad in ["qubit[2] q; while (true) { x q[0]; }",
                "qubit[2] q; foo q[0];",
                "qubit[2] q; input float[64] a; input float[64] b; rx(a * b) q[0];",
                "qubit[2] q; break;",
                "qubit[2] q; cx q[0], q[0];",
                "qubit[35] q;",
                "qubit[2] q; x q[2];",
                "bit[2] c;"]:
        with pytest.raises(QasmError):
            lower(bad)


def test_angles_combining_several_inputs_match_oracle():
    """An angle affine in several inputs reads a derived parameter (one per
    distinct combination, formed on the device before binding)."""
    src = ('OPENQASM 3.0;\ninclude "stdgates.inc";\ninput array[float[64], 3] t;\ninput float[64] s;\n'
           'qubit[3] q;\nbit[3] c;\n'
           'rx(t[0] + t[1]) q[0]; ry(2 * t[2] - t[0] + 0.3) q[1]; U(t[0] - s, t[1] + t[2], s / 2 + t[0]) q[2];\n'
           'cx q[0], q[1]; crz(t[0] + t[1]) q[1], q[2]; rz(t[1]) q[0]; cp(3 * s + t[2]) q[2], q[0];\n'
           'c = measure q;\n')
    lp = lower(src)
    assert lp.n_derived == 6 and lp.n_params == 4
    for theta in ([0.4, -1.1, 2.3, 0.7], [1.9, 0.2, -0.6, -2.5]):
        _compare(src, np.array(theta), shots=3)


def test_flag_layout_of_if_else():
    lp = lower("qubit[2] q; bit[2] c; c[0] = measure q[0]; if (c == 2) x q[1]; else h q[1];")
    ops = list(lp.instr["op"])
    assert ops == [2, 4, 4, 1, 1]
    t, e = lp.instr[1], lp.instr[2]
    assert lp.pred[int(t["pred"])]["cmp"] == 0 and lp.pred[int(e["pred"])]["cmp"] == 1
    assert int(lp.instr[3]["guard"]) == 1 << int(t["flag"])
    assert int(lp.instr[4]["guard"]) == 1 << int(e["flag"])


# ---------------------------------------------------------------------------
# Planner (host-only inspection through the C ABI)
# ---------------------------------------------------------------------------
def _qubits_of(ins):
    qs = [int(ins["q0"])]
    if int(ins["q1"]) != 0xFFFFFFFF:
        qs.append(int(ins["q1"]))
    return qs


def _check_plan(src, tile_bits=0):
    from paper_2604_11599_amd.api import plan_inspect
    lp = lower(src)
    st = plan_inspect(lp, tile_bits)
    gates = [i for i, ins in enumerate(lp.instr) if ins["op"] == 1 and ins["kind"] != 0]
    order = list(st.gate_instr[:st.n_gates])
    site_x = sorted(set(gates) - set(order))
    # every gate is planned exactly once, or folded into a measurement site (X gates only)
    assert len(order) == len(set(order))
    assert all(int(lp.instr[i]["kind"]) == 1 for i in site_x)
    # per qubit, gates keep their program order
    pos = {g: k for k, g in enumerate(order)}
    for q in range(lp.n_qubits):
        seq = [pos[i] for i in gates if i in pos and q in _qubits_of(lp.instr[i])]
        assert seq == sorted(seq)
    # register-blocked passes: every gate acts on qubits its phase holds in registers
    for k, g in enumerate(order):
        regs = st.gate_regs[k]
        if lp.n_qubits >= 4:
            assert bin(regs).count("1") == 4
            assert all(regs >> q & 1 for q in _qubits_of(lp.instr[g]))
    # every pass's tile holds the qubits of its gates
    k = 0
    for s in range(st.n_steps):
        if st.step_kind[s] == 1:
            mask = st.step_mask[s]
            assert bin(mask).count("1") == min(tile_bits or 12, lp.n_qubits)
            for g in order[k:k + st.step_count[s]]:
                for q in _qubits_of(lp.instr[g]):
                    assert mask >> q & 1
            k += st.step_count[s]
    return st


@pytest.mark.parametrize("seed", range(8))
def test_plan_invariants_random(seed):
    n = [3, 8, 13, 16, 20, 14, 17, 28][seed]
    _check_plan(W.random_dynamic_program(seed, n, n_ops=120, final_measure=True))


def test_plan_of_configs():
    st = _check_plan(W.c2_program(2, n=28, layers=40))
    assert st.n_passes <= 60
    # most brickwork phases are dense enough to run as one composed 16x16 product
    assert 0 < st.n_dense_phases <= st.n_phases and st.n_dense_phases >= st.n_phases // 2
    st = _check_plan(W.c1_program(1))
    # one pass per gate run: the whole 10-qubit state is one tile
    assert st.n_passes == 4 and st.init_step == 0
    st = _check_plan(W.c3_program(3, n=16))
    _check_plan(W.c4_ansatz(20, 6))
    _check_plan(W.brickwork_program(7, n=28, layers=6), tile_bits=10)


def test_plan_starts_with_init_when_program_starts_with_measurement():
    st = _check_plan("qubit[3] q; bit c; c = measure q[1]; h q[0];")
    assert st.init_step == 1 and st.step_kind[0] == 0 and st.step_kind[1] == 2


def test_context_close_frees_live_programs_first(monkeypatch):
    """A program must not outlive its context: Context.close frees the programs
    still alive before qsv_destroy, and a later Program.free does nothing."""
    import gc
    import weakref

    from paper_2604_11599_amd import api as api_mod
    calls = []

    class Stub:
        def qsv_destroy(self, h):
            calls.append(("destroy", h))

        def qsv_program_free(self, h):
            calls.append(("free", h))

    monkeypatch.setattr(api_mod.A, "lib", lambda: Stub())
    c = object.__new__(api_mod.Context)
    c.handle, c.device_ptrs, c._programs = 1, False, weakref.WeakSet()
    progs = []
    for h in (7, 8):
        p = object.__new__(api_mod.Program)
        p.ctx, p.handle = c, h
        c._programs.add(p)
        progs.append(p)
    c.close()
    progs[0].free()
    del progs
    gc.collect()
    assert sorted(calls[:2]) == [("free", 7), ("free", 8)] and calls[2:] == [("destroy", 1)]


@pytest.mark.parametrize("seed", range(8))
def test_lowering_of_gate_modifiers_matches_oracle(seed):
    """inv @, pow(k) @, ctrl @, negctrl @ lower to standard gates (controlled U
    and SX by decomposition); the oracle applies them by definition."""
    _compare(W.modifier_program(seed, 3 + seed % 3, 30), shots=2)


@pytest.mark.parametrize("seed", range(10))
def test_lowering_of_logical_conditions_matches_oracle(seed):
    """`&&`, `||` and `!` in if conditions lower to disjoint flag guards (the
    body once per way the condition holds); the oracle evaluates them directly."""
    _compare(W.logic_program(seed, 2 + seed % 4, 30), shots=4)


def test_logical_condition_guards_are_disjoint():
    """Every shot runs the then-body at most once: a condition that holds in
    several ways still flips the target qubit exactly once."""
    head = 'OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[4] q;\nbit[3] c;\nbit t;\n'
    for pre in ("", "x q[0];", "x q[0]; x q[1];", "x q[0]; x q[1]; x q[2];", "x q[2];"):
        src = (head + pre + "c[0] = measure q[0]; c[1] = measure q[1]; c[2] = measure q[2];"
               "if (c[0] || c[1] || c[2] || c == 7) x q[3]; t = measure q[3];")
        _compare(src, shots=1)


@pytest.mark.parametrize("seed", range(8))
def test_lowering_of_classical_assignment_matches_oracle(seed):
    """c[i] = <condition> and c = <integer> lower to set / clear bit events
    after the condition's predicates; the oracle assigns directly."""
    _compare(W.logic_program(100 + seed, 2 + seed % 4, 40, assign=True), shots=4)


def test_classical_assignment_forms():
    head = ('OPENQASM 3.0;\ninclude "stdgates.inc";\nconst int k = 6;\nqubit[4] q;\nbit[3] c;\n'
            'bit[3] d;\nbit t;\n')
    for pre in ("", "x q[0];", "x q[1]; x q[2];", "x q[0]; x q[1]; x q[2];"):
        meas = "c[0] = measure q[0]; c[1] = measure q[1]; c[2] = measure q[2];"
        for body in ("d = c; c = 5;", "c[2] = c[0] && !c[1] || !c[0] && c[1]; if (c[2]) x q[3]; t = measure q[3];",
                     "c[0] = !c[0] && c[1]; d[1] = c >= 3;", "c = k; d = 0b101; d[0] = c[1];"):
            _compare(head + pre + meas + body, shots=1)
        # integer semantics: a condition into a whole register, a negative value,
        # a copy between widths
        for body in ("c = d[0] && d[1];", "c = -1;", "c = t;", "d = c + 3;"):
            _compare(head + pre + meas + body, shots=1)
    # not integers, or not classical
    for bad in ("c = 1.5;", "c = q;", "c = c + q[0];"):
        with pytest.raises(QasmError):
            lower(head + bad)


CLASSICAL_PROGRAMS = [
    # register arithmetic and bitwise operators, stored on the device
    "d = c + 1; t = c > d; int[8] x = c * 3 - d; uint[5] u = (c << 2) | d; x >>= 1; u ^= x;",
    # register-versus-register comparisons and expressions in conditions
    "if (c == d) x q[3]; if (c < d && (c & 1) == 0) h q[3]; if (!(c + d > 4) || c ^ d) x q[3]; t = measure q[3];",
    # a counter over a bounded loop with feed-forward on the count
    "uint[4] n = 0; for uint i in [0:2] { h q[i]; c[i] = measure q[i]; if (c[i]) n += 1; } "
    "if (n >= 2) x q[3]; t = measure q[3]; d = n;",
    # signed variables, division and modulo, shifts past the width
    "int[6] y = -5; y = y / 2 + c % 3; int[16] z = (y << 3) >> 1; uint[3] w = z; if (y < 0) x q[3]; t = measure q[3];",
    # compound assignments on bits and variables; constants fold
    "bool b = c[0]; b |= c[1]; c[2] ^= b; int[8] m = k * 4 + 1; m -= c; if (m % 2 == 1) x q[3]; t = measure q[3];",
]


@pytest.mark.parametrize("body", CLASSICAL_PROGRAMS)
def test_lowering_of_classical_expressions_matches_oracle(body):
    """Integer variables, register arithmetic, register-versus-register
    comparisons and computed conditions: the lowered stream (expression code
    stored by CSTORE, EXPR predicates) equals the oracle's tree walk."""
    head = ('OPENQASM 3.0;\ninclude "stdgates.inc";\nconst int k = 6;\nqubit[4] q;\nbit[3] c;\n'
            'bit[3] d;\nbit t;\n')
    for pre in ("", "x q[0];", "x q[1]; x q[2];", "x q[0]; x q[2];", "h q[0]; h q[1]; h q[2];"):
        meas = "c[0] = measure q[0]; c[1] = measure q[1]; c[2] = measure q[2]; d = c;"
        _compare(head + pre + meas + body, shots=3)


MULTI_CONTROL = [
    "ctrl @ cx q[0], q[1], q[2];", "ctrl(2) @ x q[0], q[1], q[2];", "ctrl @ ctrl @ U(0.4, 1.2, -0.7) q[0], q[1], q[2];",
    "negctrl @ ctrl @ h q[3], q[0], q[2];", "ctrl(2) @ rz(th[0]) q[4], q[1], q[0];", "ctrl @ swap q[0], q[1], q[2];",
    "ctrl(3) @ x q[0], q[1], q[2], q[3];", "ctrl @ cp(0.7) q[2], q[0], q[1];", "ctrl @ crx(th[1]) q[3], q[4], q[0];",
    "ctrl @ cy q[1], q[2], q[3];", "ctrl @ cz q[4], q[2], q[0];", "ctrl @ ch q[0], q[3], q[1];",
    "ctrl @ cry(0.9) q[1], q[4], q[2];", "ctrl @ crz(-1.1) q[2], q[0], q[3];", "inv @ ctrl(2) @ sx q[0], q[1], q[2];",
    "ctrl @ inv @ ctrl @ t q[0], q[1], q[2];", "ctrl @ pow(2) @ ctrl @ sx q[3], q[1], q[2];",
    "negctrl(2) @ y q[0], q[1], q[4];", "ctrl(2) @ U(th[0], 0.2, th[1]) q[3], q[0], q[1];",
]


@pytest.mark.parametrize("body", MULTI_CONTROL)
def test_multi_controlled_gates_match_oracle(body):
    """Several controls and controls on two-qubit gates lower exactly to
    one-qubit gates and CX (two-qubit gates through their CX decomposition,
    each controlled CX as a Toffoli); the oracle builds the controlled matrix
    by definition."""
    src = ('OPENQASM 3.0;\ninclude "stdgates.inc";\ninput array[float[64], 2] th;\nqubit[5] q;\n'
           "U(0.3, 1.1, -0.4) q[0]; U(1.3, -0.2, 0.9) q[1]; U(2.1, 0.5, 0.1) q[2]; U(0.7, 2.2, -1.3) q[3];"
           "U(1.9, -0.8, 0.6) q[4];\n" + body + "\n")
    _compare(src, theta=np.array([0.37, -1.21]), shots=1)


def test_gate_modifier_limits_are_reported():
    for body in ("pow @ x q[0];", "pow(0.5) @ x q[0];", "ctrl(0) @ x q[0];", "ctrl @ x q[0];"):
        with pytest.raises(QasmError):
            lower('OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[3] q;\n' + body + "\n")


# ---------------------------------------------------------------------------
# Depolarizing slots: lowering with noise == the oracle with noise, shot by shot
# ---------------------------------------------------------------------------
def _compare_noisy(src, p=0.2, shots=4, seed=13):
    lp = lower(src, noise=True)
    assert not lp.is_unitary and len(lp.noise) == int(np.sum(lp.instr["op"] == 9))
    hit = 0
    for shot in range(shots):
        o = sim.run_shot(src, seed=seed, shot=shot, depolarizing=p)
        psi, bits, record = ir_interp.run(lp, (), seed=seed, shot=shot, depolarizing=p)
        assert bits == o.cbits and record == o.record
        assert np.max(np.abs(psi - o.psi)) < 1e-13
        hit += len(o.noise_events)
    return hit


@pytest.mark.parametrize("seed", range(10))
def test_noise_slots_match_oracle_random_dynamic(seed):
    assert _compare_noisy(W.random_dynamic_program(seed, 2 + seed % 5, n_ops=40, final_measure=True)) > 0


@pytest.mark.parametrize("seed", range(4))
def test_noise_slots_match_oracle_modifiers_and_logic(seed):
    """Modified gates (one draw per operand, controls included, after the whole
    decomposition) and bodies emitted once per guard of a logical condition
    (each copy carries the same draws)."""
    _compare_noisy(W.modifier_program(seed, 3 + seed % 3, 30), shots=2)
    _compare_noisy(W.logic_program(seed, 2 + seed % 4, 30), shots=3)


def test_noise_slots_loops_custom_gates_and_broadcast():
    """Draws named by statement, loop ordinals (nested, with break and
    continue), application index of a broadcast and operand; a custom gate
    call draws once per operand after its body."""
    src = ('OPENQASM 3.0;\ninclude "stdgates.inc";\ngate g(a) x, y { rx(a) x; cx x, y; ry(a) y; }\n'
           'qubit[3] q;\nbit[3] c;\nbit f;\n'
           'for int i in [0:3] { h q[0]; f = measure q[0]; if (f == 1) continue; '
           'for int j in [1:2] { g(0.3) q[j], q[0]; h q[2]; c[2] = measure q[2]; if (c[2] == 1) break; } }\n'
           'x q;\nc = measure q;\n')
    assert _compare_noisy(src, p=0.3, shots=6) > 0
    # without a positive rate the slots change nothing
    lp = lower(src, noise=True)
    for shot in range(3):
        o = sim.run_shot(src, seed=2, shot=shot)
        psi, bits, record = ir_interp.run(lp, (), seed=2, shot=shot)
        assert bits == o.cbits and np.max(np.abs(psi - o.psi)) < 1e-13


def test_noise_slot_validation_on_the_host():
    """The planner takes noise slots as one-qubit dense gates (one matrix slot
    each) and rejects slots whose counter index or gate kind is out of range."""
    from paper_2604_11599_amd import QsvError
    from paper_2604_11599_amd.api import plan_inspect
    src = 'OPENQASM 3.0;\ninclude "stdgates.inc";\nqubit[3] q;\nbit[3] c;\nh q[0];\ncx q[0], q[1];\nc = measure q;\n'
    plain, noisy = plan_inspect(lower(src)), plan_inspect(lower(src, noise=True))
    assert noisy.n_gates == plain.n_gates + 3 and not noisy.is_unitary
    lp = lower(src, noise=True)
    bad = lower(src, noise=True)
    k = int(np.flatnonzero(bad.instr["op"] == 9)[0])
    bad.instr["pred"][k] = len(bad.noise)
    with pytest.raises(QsvError):
        plan_inspect(bad)
    bad = lower(src, noise=True)
    bad.instr["kind"][k] = 4
    with pytest.raises(QsvError):
        plan_inspect(bad)
    assert plan_inspect(lp).n_gates == noisy.n_gates
