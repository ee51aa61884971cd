"""The allocation-free entry point (mpc_run_noalloc, static device scratch)
against the handle-based path (mpc_create + set_state + set_step + step +
get_state) on the same inputs: two calls in a row, the second on a smaller
box, then a box too large for the scratch.  Bar as for every FP64 parity
test: positions bit-identical, velocities within e <= 1e-12."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

DEG = math.pi / 180.0


@pytest.fixture(scope="module")
def mpc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_15236_amd as m
    m.lib()
    return m


def box_of(L, **kw):
    b = dict(L=tuple(L), h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=10.0, seed=7,
             mbs=True, walls=False, g=(0.0, 0.0, 0.0))
    b.update(kw)
    return b


def handle_path(mpc, box, R, x, v, t0, nsteps):
    with mpc.Sim(box, form="fp64", reorder_every=R) as sim:
        sim.set_state(x, v)
        sim.set_step(t0)
        sim.step(nsteps)
        return sim.get_state()


def noalloc_path(mpc, box, R, x, v, t0, nsteps):
    import torch
    p = mpc.make_params(box, "fp64", reorder_every=R)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    vd = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    st = torch.cuda.current_stream().cuda_stream
    mpc.run_noalloc(p, xd.data_ptr(), vd.data_ptr(), x.shape[1], t0, nsteps, st)
    torch.cuda.synchronize()
    return xd.cpu().numpy(), vd.cpu().numpy()


def compare(xa, va, xb, vb, box):
    np.testing.assert_array_equal(xa, xb)
    floor = math.sqrt(box["kT"] / box["mass"])
    e = np.linalg.norm(va - vb, axis=0) / np.maximum(np.linalg.norm(vb, axis=0), floor)
    print(f"max e = {e.max():.3e} (bit-identical: {np.array_equal(va, vb)})", flush=True)
    assert e.max() <= 1e-12


@pytest.mark.parametrize("case", [
    # L, extra box keys, R, t0, steps
    ((14, 11, 9), {}, 3, 5, 4),
    ((9, 7, 6), {"walls": True, "g": (1e-3, 0.0, 0.0)}, 0, 11, 3),   # smaller, second call
])
def test_noalloc_matches_handle_path(mpc, case):
    L, kw, R, t0, nsteps = case
    box = box_of(L, **kw)
    x, v = synth.box_state(L, seed=sum(L))
    print(f"case noalloc L={L} {kw} R={R} t0={t0} steps={nsteps}", flush=True)
    xa, va = noalloc_path(mpc, box, R, x, v, t0, nsteps)
    xb, vb = handle_path(mpc, box, R, x, v, t0, nsteps)
    compare(xa, va, xb, vb, box)


def test_noalloc_two_calls_in_a_row(mpc):
    """Back-to-back calls share the scratch: the second (smaller) call must not
    see anything the first left behind."""
    big = box_of((16, 13, 12), seed=3)
    small = box_of((7, 6, 5), seed=4, mbs=False)
    xb, vb = synth.box_state(big["L"], seed=41)
    xs, vs = synth.box_state(small["L"], seed=42)
    out_big = noalloc_path(mpc, big, 2, xb, vb, 0, 5)
    out_small = noalloc_path(mpc, small, 1, xs, vs, 9, 2)
    compare(*out_big, *handle_path(mpc, big, 2, xb, vb, 0, 5), big)
    compare(*out_small, *handle_path(mpc, small, 1, xs, vs, 9, 2), small)


def test_noalloc_limits(mpc):
    import torch
    # a box whose workspace exceeds the 256 MiB scratch is refused before any launch
    big = box_of((160, 160, 160))
    p = mpc.make_params(big, "fp64")
    assert mpc.workspace_bytes(p) > 256 << 20
    xd = torch.zeros(3, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(mpc.MPCError) as e:
        mpc.run_noalloc(p, xd.data_ptr(), xd.data_ptr(), 40960000, 0, 1, 0)
    assert e.value.code == mpc.ERANGE
    # positions outside the box are refused (checked on the device)
    box = box_of((6, 6, 6))
    x, v = synth.box_state(box["L"], seed=5)
    x[0, 3] = 6.5
    with pytest.raises(mpc.MPCError) as e:
        noalloc_path(mpc, box, 0, x, v, 0, 1)
    assert e.value.code == mpc.EINVAL
    # FP32 / split forms are not offered here
    with pytest.raises(mpc.MPCError) as e:
        mpc.run_noalloc(mpc.make_params(box, "split"), xd.data_ptr(), xd.data_ptr(),
                        2160, 0, 1, 0)
    assert e.value.code == mpc.EINVAL
