"""The C-ABI library loads on the CPU host and exports every declared call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpc.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(mpc_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_calls():
    names = declared_symbols()
    for must in ["mpc_workspace_bytes", "mpc_create", "mpc_step", "mpc_observables",
                 "mpc_set_state", "mpc_get_state", "mpc_get_binning", "mpc_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2406_15236_amd as m
    if not os.path.exists(m.LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(m.LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert sorted(m.SYMBOLS) == declared_symbols()


def test_workspace_planning_and_validation_on_host():
    """Parameter checks and the workspace size need no GPU."""
    import paper_2406_15236_amd as m
    import synth
    if not os.path.exists(m.LIB):
        pytest.skip("library not built")
    c1 = synth.config("C1")
    p = m.make_params(c1, "fp64")
    nb = m.workspace_bytes(p)
    n = 40960
    assert nb >= 2 * 48 * n + 8 * n
    # FP32 and split need less state
    assert m.workspace_bytes(m.make_params(c1, "fp32")) < nb
    bad = m.make_params(dict(c1, h=-0.1))
    with pytest.raises(m.MPCError) as e:
        m.workspace_bytes(bad)
    assert e.value.code == m.EINVAL
    big = m.make_params(dict(c1, L=(2048, 2048, 1024)))  # 4.3e10 particles
    with pytest.raises(m.MPCError) as e:
        m.workspace_bytes(big)
    assert e.value.code == m.ERANGE
    split_big = m.make_params(dict(c1, L=(4096, 8, 8), density=1.0), "split")
    with pytest.raises(m.MPCError) as e:
        m.workspace_bytes(split_big)
    assert e.value.code == m.ERANGE
    # degenerate inputs: a box whose density rounds to no particle, zero or
    # negative density, an axis of zero cells
    for degenerate in (dict(c1, L=(4, 4, 4), density=1e-3), dict(c1, density=0.0),
                       dict(c1, density=-1.0), dict(c1, L=(16, 0, 16))):
        with pytest.raises(m.MPCError) as e:
            m.workspace_bytes(m.make_params(degenerate))
        assert e.value.code == m.EINVAL
    # the smallest box: one cell
    assert m.workspace_bytes(m.make_params(dict(c1, L=(1, 1, 1)))) > 0
    mixed = [m.make_params(c1, "fp64"), m.make_params(c1, "fp32")]
    with pytest.raises(m.MPCError) as e:
        m.workspace_bytes(mixed)
    assert e.value.code == m.EINVAL
    # batched: sizes add up
    boxes = synth.batch_boxes(4, lmin=16, lmax=20)
    tot = m.workspace_bytes([m.make_params(b) for b in boxes])
    assert tot > max(m.workspace_bytes(m.make_params(b)) for b in boxes)


def test_amc_flag_validation_on_host():
    """SRD+a (MPC_AMC) is accepted for periodic boxes and slip walls, with or
    without the thermostat, and refused with no-slip walls."""
    import paper_2406_15236_amd as m
    import synth
    if not os.path.exists(m.LIB):
        pytest.skip("library not built")
    c1 = synth.config("C1")
    assert m.workspace_bytes(m.make_params(dict(c1, amc=True))) > 0
    assert m.workspace_bytes(m.make_params(dict(c1, amc=True, mbs=True))) > 0
    with pytest.raises(m.MPCError) as e:
        m.workspace_bytes(m.make_params(dict(c1, amc=True, walls=True)))
    assert e.value.code == m.EINVAL
    assert m.workspace_bytes(m.make_params(dict(c1, amc=True, walls=True, slip=True))) > 0
    with pytest.raises(m.MPCError) as e:
        m.workspace_bytes(m.make_params(c1, flags=16))
    assert e.value.code == m.EINVAL


def test_boundary_parameter_validation_on_host():
    """Slip walls need walls; wall_u needs no-slip walls; le_u needs a periodic
    box; non-finite wall_u or le_u are refused."""
    import paper_2406_15236_amd as m
    import synth
    if not os.path.exists(m.LIB):
        pytest.skip("library not built")
    c5 = dict(synth.config("C5"), L=(16, 16, 8))
    c1 = synth.config("C1")
    assert m.workspace_bytes(m.make_params(dict(c5, slip=True))) > 0
    assert m.workspace_bytes(m.make_params(dict(c5, uwall=0.2))) > 0
    assert m.workspace_bytes(m.make_params(dict(c1, le_u=0.5, amc=True, fixed=True))) > 0
    for bad in (dict(c1, slip=True), dict(c5, slip=True, uwall=0.1), dict(c1, uwall=0.1),
                dict(c5, le_u=0.5), dict(c1, le_u=float("nan")), dict(c5, uwall=float("inf"))):
        with pytest.raises(m.MPCError) as e:
            m.workspace_bytes(m.make_params(bad))
        assert e.value.code == m.EINVAL
