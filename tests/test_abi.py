"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/sv.h declares, validates gate arguments, and the
fusion planner (host only) reproduces the circuit it fuses."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2511_19291_amd import circuits as Cc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def svmod():
    from paper_2511_19291_amd import sv
    sv.lib()
    return sv


def test_header_declares_entry_points():
    names = _declared()
    for required in ["sv_alloc", "sv_apply_gate", "sv_apply_fused", "sv_expval_pauli", "sv_adjoint_grad",
                     "sv_run", "sv_batch_plan_create", "sv_batch_launch"]:
        assert required in names


def test_library_exports_every_declared_symbol(svmod):
    L = svmod.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(svmod):
    L = svmod.lib()
    for st in range(0, 9):
        assert L.sv_status_string(st)
    assert L.sv_status_string(99) == b"unknown status"


@pytest.mark.parametrize("n,seed", [(3, 1), (6, 2), (9, 3)])
def test_fusion_plan_reproduces_circuit(svmod, n, seed):
    """The host fusion planner's blocks, applied in order by the oracle, give
    the oracle's gate-by-gate state (the planner only regroups gates)."""
    import oracle
    circ = Cc.random_circuit(n, 120, seed)
    for max_k in (3, 4, 5):
        if max_k < 5 and any(len(op.qubits()) > max_k for op in circ.ops):
            continue
        blocks = svmod.fuse_plan(circ, max_k)
        assert all(len(t) <= max_k for t, _ in blocks)
        psi = oracle.basis_state(n)
        for t, m in blocks:
            oracle.apply_matrix(psi, n, m, list(t))
        np.testing.assert_allclose(psi, oracle.run(circ), atol=1e-12)


@pytest.mark.parametrize("name", ["qft", "ring", "hea", "brickwork", "ghz"])
def test_fusion_plan_reproduces_structured_circuits(svmod, name):
    """The same check on structured circuits, where the frontier planner and
    the open-block planner take turns at giving the fewest blocks."""
    import oracle
    circ = {"qft": lambda: Cc.qft(9, 77), "ring": lambda: Cc.rxry_ring(9, 3, 2), "hea": lambda: Cc.hea_ladder(9, 3, 4),
            "brickwork": lambda: Cc.brickwork_u3_cz(10, 6, 5), "ghz": lambda: Cc.ghz(10)}[name]()
    for max_k in (2, 3, 5):
        blocks = svmod.fuse_plan(circ, max_k)
        assert all(len(t) <= max_k for t, _ in blocks)
        psi = oracle.basis_state(circ.n)
        for t, m in blocks:
            oracle.apply_matrix(psi, circ.n, m, list(t))
        np.testing.assert_allclose(psi, oracle.run(circ), atol=1e-12)


def test_fusion_plan_brickwork_block_count(svmod):
    """The brickwork workloads fuse into far fewer 5-qubit sweeps: 890 gates
    at 30 qubits -> 52 blocks, 950 at 32 -> 56 (the frontier planner; the
    open-block planner alone gives 72 and 80)."""
    for n, seed, most in ((30, 2, 52), (32, 3, 56)):
        blocks = svmod.fuse_plan(Cc.brickwork_u3_cz(n, 20, seed), 5)
        assert len(blocks) <= most
        assert sum(len(t) == 5 for t, _ in blocks) >= 0.8 * len(blocks)


def test_fusion_plan_rejects_bad_input(svmod):
    circ = Cc.random_circuit(4, 10, 1)
    with pytest.raises(svmod.SvError):
        svmod.fuse_plan(circ, 7)
    bad = Cc.Circuit(4, [Cc.Op("x", (4,))], np.zeros(0))
    with pytest.raises(svmod.SvError):
        svmod.fuse_plan(bad, 5)


@pytest.mark.parametrize("n,targets,controls,code", [
    (4, [0], [], 0), (4, [3, 0], [1, 2], 0), (4, [4], [], 2), (4, [-1], [], 2), (4, [1], [1], 3),
    (4, [0, 0], [], 3), (4, [0, 1, 2], [], 4), (5, [0], [1, 2, 3, 4], 4), (2, [0, 1], [], 0),
    (2, [0], [1], 0), (1, [0], [], 0), (40, [0], [], 1), (0, [0], [], 1),
])
def test_gate_validation_host_only(svmod, n, targets, controls, code):
    L = svmod.lib()
    ta = (C.c_int * max(1, len(targets)))(*targets)
    ca = (C.c_int * max(1, len(controls)))(*controls)
    assert L.sv_check_gate(n, ta, len(targets), ca, len(controls)) == code


def test_batch_config_default_and_validation_host_only(svmod):
    """The default launch shape, and out-of-range shapes rejected before any
    device work (no GPU needed)."""
    assert svmod.default_batch_config() == {"tile_bits": 14, "threads": 512, "reg_min_bits": 12, "wg_per_cu": 0,
                                            "phase_mode": 1, "fuse_min_gates": 3, "run_bits": 3}
    circ = Cc.ghz(3)
    table = svmod.OpTable(circ.ops)
    ops_arr = (C.POINTER(svmod.SvOp) * 1)(C.cast(table.arr, C.POINTER(svmod.SvOp)))
    bad = [(9, 1024, 12, 0, 1, 3, 4), (15, 1024, 12, 0, 1, 3, 4), (12, 128, 12, 0, 1, 3, 4),
           (12, 256, 3, 0, 1, 3, 4), (12, 256, 16, 0, 1, 3, 4), (12, 256, 12, -1, 1, 3, 4),
           (12, 256, 12, 17, 1, 3, 4), (12, 256, 12, 0, 3, 3, 4), (12, 256, 12, 0, -1, 3, 4),
           (12, 256, 12, 0, 1, 0, 4), (12, 256, 12, 0, 2, 65, 4), (12, 256, 12, 0, 1, 3, 2),
           (12, 256, 12, 0, 1, 3, 7), (10, 256, 10, 0, 1, 3, 6)]
    for cfg in bad:
        h = C.c_void_p()
        st = svmod.lib().sv_batch_plan_create_ex(1, svmod._iarr([3]), ops_arr, svmod._iarr([table.n]),
                                                 svmod._iarr([0]), C.byref(svmod.SvBatchConfig(*cfg)), None,
                                                 C.byref(h))
        assert st == 1 and not h.value, cfg
        assert b"must be" in svmod.lib().sv_last_error()


def test_error_hooks_reject_null_state_host_only(svmod):
    """The sticky-error query and the testing hook validate their state
    argument like every other entry point (no GPU needed)."""
    L = svmod.lib()
    f = C.c_int(7)
    assert L.sv_state_failed(None, C.byref(f)) == 1 and f.value == 7
    assert L.sv_inject_hip_error(None) == 1
    assert b"null state" in L.sv_last_error()
