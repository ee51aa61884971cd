"""Parity at full size: the 256^3 box with 10 particles per cell
(167,772,160 particles), thermostat on, FP64, reorder interval 20, in the
launch configuration the benchmark uses, one step from a synthetic state.

The same box with the angular-momentum-conserving collision SRD+a (Eqs. 3-4,
thermostat on) is checked the same way.

Post-stream positions, cell keys, the sort permutation and the offsets are
compared with the oracle for every particle; velocities (e <= 1e-12) for the
particles of a random sample of cells, which the oracle collides on their own
(an offset table in which only the sampled cells are occupied).
"""
import math
import time

import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_15236_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("t0,amc", [(19, False), (19, True)])
def test_c2_full_size_one_step(mpc, t0, amc):
    """amc: the same box and thermostat with the collision SRD+a (Eqs. 3-4)."""
    box = synth.config("C2")
    if amc:
        box = dict(box, amc=True)
    L = box["L"]
    t_start = time.time()
    x, v = synth.box_state(L, seed=2024)
    n = x.shape[1]
    print(f"C2 full size (amc={amc}): n = {n}, state made in {time.time() - t_start:.1f} s",
          flush=True)
    with mpc.Sim(box, form="fp64", reorder_every=20) as sim:
        sim.set_state(x, v)
        sim.set_step(t0)
        sim.step(1)
        xg, vg = sim.get_state()
        kg, pg, og = sim.get_binning()
        print(f"GPU step and transfers done at {time.time() - t_start:.1f} s, tiling "
              f"{sim.get_tiling()}", flush=True)
    p = orc.Params(L=L, h=box["h"], alpha=box["alpha"], kT=box["kT"], mass=box["mass"],
                   density=box["density"], seed=box["seed"], mbs=box["mbs"], amc=amc)
    xs, vs, _ = orc.stream(p, x, v)
    del x
    ko = orc.keys(p, t0, xs)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    np.testing.assert_array_equal(og, oo)
    np.testing.assert_array_equal(pg, po)
    del kg, ko, pg
    renumber = (t0 + 1) % 20 == 0
    # the GPU state is in the caller's order after the step: renumbered to
    # cell order on a reorder step
    order = po if renumber else np.arange(n, dtype=np.uint32)
    np.testing.assert_array_equal(xg, xs[:, order])
    print(f"positions, keys, permutation, offsets equal at {time.time() - t_start:.1f} s",
          flush=True)
    # velocities on sampled cells
    rng = np.random.default_rng(7)
    cells = np.sort(rng.choice(p.ncells, size=2000, replace=False))
    counts = (oo[cells + 1] - oo[cells]).astype(np.int64)
    off_s = np.zeros(p.ncells + 1, dtype=np.uint32)
    cnt_all = np.zeros(p.ncells, dtype=np.int64)
    cnt_all[cells] = counts
    off_s[1:] = np.cumsum(cnt_all).astype(np.uint32)
    members = np.concatenate([po[oo[c]:oo[c + 1]] for c in cells]).astype(np.int64)
    vsub = np.ascontiguousarray(vs[:, members])
    perm_s = np.arange(members.size, dtype=np.uint32)
    xsub = np.ascontiguousarray(xs[:, members]) if amc else None
    vo = orc.collide(p, t0, vsub, perm_s, off_s, x=xsub)
    if renumber:
        inv = np.empty(n, dtype=np.int64)
        inv[po] = np.arange(n)
        gidx = inv[members]
    else:
        gidx = members
    vgs = vg[:, gidx]
    floor = math.sqrt(box["kT"] / box["mass"])
    e = np.linalg.norm(vgs - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), floor)
    print(f"velocities on {cells.size} cells ({members.size} particles): max e = {e.max():.3e}"
          f" (total {time.time() - t_start:.1f} s)", flush=True)
    if amc:
        # omega = I^-1 dL: rounding differences scale with cond(I) of the cell
        y = xsub + orc.shift(p, t0)[:, None]
        fr = y - np.floor(y)
        cond = np.ones(members.size)
        for c0, c1 in zip(off_s[cells], off_s[cells + 1]):
            if c1 - c0 >= 3:
                r = fr[:, c0:c1] - fr[:, c0:c1].mean(axis=1, keepdims=True)
                cond[c0:c1] = np.linalg.cond((r * r).sum() * np.eye(3) - r @ r.T)
        assert np.all(e <= 1e-12 + 64 * 2.0 ** -52 * cond)
    else:
        assert e.max() <= 1e-12
