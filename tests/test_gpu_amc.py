"""GPU parity of the angular-momentum-conserving collision SRD+a (Eqs. 3-4).

One step from the same state, HIP path through the C ABI against the oracle:
  * FP64 form: positions, keys, permutation and offsets bit-identical;
    velocities within e <= 1e-12 + 64 eps cond(I_c) per particle (e as in the
    other parity tests).  omega = I^-1 dL is as well conditioned as the cell's
    inertia tensor I_c: the two sides sum I and dL in different orders (the
    GPU splits each cell over two lanes), so their rounding differences are
    amplified by cond(I_c).  A cell of two uses the pseudo-inverse (cond 1).
  * FP32 and split forms: the oracle collides the GPU's post-stream state;
    e <= 2e-6.
  * With the thermostat (MPC_MBS) the corrected relative velocities are
    scaled to the drawn energy; the same bars apply.
  * Invariant at any size: per cell, momentum and angular momentum about the
    centre of mass are unchanged by the GPU's collision.
"""
import math

import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu

DEG = math.pi / 180.0
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def mpc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_15236_amd as m
    m.lib()
    return m


def box_of(L, seed=1, density=10.0, g=(0.0, 0.0, 0.0), **kw):
    b = dict(L=tuple(L), h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=density,
             seed=seed, mbs=False, walls=False, amc=True, g=tuple(g))
    b.update(kw)
    return b


def oparams(box):
    return orc.Params(L=box["L"], h=box["h"], alpha=box["alpha"], kT=box["kT"],
                      mass=box["mass"], density=box["density"], seed=box["seed"],
                      mbs=box["mbs"], amc=True, g=box["g"])


def rel_err(vg, vo, box):
    floor = math.sqrt(box["kT"] / box["mass"])
    return np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), floor)


def frame(p, t, xs):
    y = xs + orc.shift(p, t)[:, None]
    return y - np.floor(y)


def cell_cond(key, off, perm, fr):
    """cond(I_c) of every particle's cell (1 for cells of one or two)."""
    n = key.size
    cond = np.ones(n)
    for c in np.nonzero(np.diff(off) >= 3)[0]:
        idx = perm[off[c]:off[c + 1]]
        r = fr[:, idx] - fr[:, idx].mean(axis=1, keepdims=True)
        inertia = (r * r).sum() * np.eye(3) - r @ r.T
        cond[idx] = np.linalg.cond(inertia)
    return cond


AMC_CASES = [
    # L, density, gravity, R, t0, thermostat
    ((16, 16, 16), 10.0, (0, 0, 0), 0, 0, False),
    ((16, 16, 16), 10.0, (0, 0, 0), 0, 0, True),
    ((13, 9, 11), 10.0, (0, 0, 0), 1, 3, False),         # ragged tiles, sorted output
    ((13, 9, 11), 10.0, (0, 0, 0), 3, 2, True),          # reorder step of R = 3
    ((12, 10, 8), 10.0, (2e-3, 0, -1e-3), 3, 2, True),   # gravity
    ((10, 10, 10), 2.0, (0, 0, 0), 0, 5, False),         # many cells of one, two, three
    ((10, 10, 10), 2.0, (0, 0, 0), 1, 6, True),
    ((6, 5, 7), 60.0, (0, 0, 0), 1, 1, True),            # tiles in several passes
    ((1, 1, 1), 10.0, (0, 0, 0), 1, 2, True),            # a single cell
    ((2, 3, 1), 10.0, (0, 0, 0), 0, 3, False),           # one and two cells per axis
]


@pytest.mark.parametrize("L,density,g,R,t0,mbs", AMC_CASES)
def test_amc_fp64_one_step(mpc, L, density, g, R, t0, mbs):
    box = box_of(L, seed=7 + t0, density=density, g=g, mbs=mbs)
    x, v = synth.box_state(L, density=density, seed=13 + t0, kT=0.8 if mbs else 1.0)
    print(f"case amc fp64 L={L} density={density} R={R} t0={t0} mbs={mbs}", flush=True)
    with mpc.Sim(box, form="fp64", reorder_every=R) as sim:
        if density > 30:
            sim.set_tiling(32, 0, 0)
        sim.set_state(x, v)
        sim.set_step(t0)
        sim.step(1)
        xg, vg = sim.get_state()
        kg, pg, og = sim.get_binning()
    p = oparams(box)
    sorted_out = R > 0 and (t0 + 1) % R == 0
    xo, vo, ko, po, oo = orc.step(p, t0, x, v, reorder=sorted_out, binning=True)
    np.testing.assert_array_equal(kg, ko)
    np.testing.assert_array_equal(pg, po)
    np.testing.assert_array_equal(og, oo)
    np.testing.assert_array_equal(xg, xo)
    xs, _, _ = orc.stream(p, x, v)
    cond = cell_cond(ko, oo, po, frame(p, t0, xs))
    if sorted_out:
        cond = cond[po]
    e = rel_err(vg, vo, box)
    tol = 1e-12 + 64 * EPS * cond
    print(f"amc fp64: max e = {e.max():.3e}, max e/tol = {(e / tol).max():.3f}, "
          f"max cond = {cond.max():.3e}")
    assert np.all(e <= tol)


def test_amc_batched_boxes(mpc):
    """SRD+a with the thermostat on a batch of uneven boxes (a single-cell box
    among them, different angles, temperatures and gravity per box): each box
    equals its own oracle step, with the cond(I_c) bar."""
    shapes = [(9, 7, 8), (1, 1, 1), (12, 5, 6), (4, 3, 2)]
    boxes = [box_of(L, seed=60 + i, mbs=True, alpha=(100.0 + 15.0 * i) * DEG,
                    kT=0.7 + 0.2 * i, g=(1e-3 * i, 0.0, 0.0)) for i, L in enumerate(shapes)]
    states = [synth.box_state(b["L"], density=b["density"], kT=b["kT"], seed=300 + i)
              for i, b in enumerate(boxes)]
    t0 = 4
    with mpc.Sim(boxes, form="fp64", reorder_every=5) as sim:
        for i, (x, v) in enumerate(states):
            sim.set_state(x, v, box=i)
        sim.set_step(t0)
        sim.step(1)
        outs = [sim.get_state(box=i) for i in range(len(boxes))]
        bins = [sim.get_binning(box=i) for i in range(len(boxes))]
    sorted_out = (t0 + 1) % 5 == 0
    for i, b in enumerate(boxes):
        x, v = states[i]
        p = oparams(b)
        xo, vo, ko, po, oo = orc.step(p, t0, x, v, reorder=sorted_out, binning=True)
        np.testing.assert_array_equal(bins[i][0], ko)
        np.testing.assert_array_equal(bins[i][1], po)
        np.testing.assert_array_equal(bins[i][2], oo)
        np.testing.assert_array_equal(outs[i][0], xo)
        xs, _, _ = orc.stream(p, x, v)
        cond = cell_cond(ko, oo, po, frame(p, t0, xs))
        if sorted_out:
            cond = cond[po]
        e = rel_err(outs[i][1], vo, b)
        tol = 1e-12 + 64 * EPS * cond
        print(f"box {i} {b['L']}: max e = {e.max():.3e}, max e/tol = {(e / tol).max():.3f}")
        assert np.all(e <= tol), i


@pytest.mark.parametrize("form,mbs", [("fp32", False), ("split", False), ("fp32", True),
                                      ("split", True)])
def test_amc_reduced_precision_one_step(mpc, form, mbs):
    L = (16, 12, 10)
    box = box_of(L, seed=9, mbs=mbs)
    x, v = synth.box_state(L, seed=21)
    t0 = 4
    print(f"case amc form={form} mbs={mbs}", flush=True)
    with mpc.Sim(box, form=form) as sim:
        sim.set_state(x, v)
        _, v0 = sim.get_state()
        sim.set_step(t0)
        sim.step(1)
        x1, v1 = sim.get_state()
        kg, pg, og = sim.get_binning()
    p = oparams(box)
    ko = orc.keys(p, t0, x1)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    np.testing.assert_array_equal(pg, po)
    np.testing.assert_array_equal(og, oo)
    vo = orc.collide(p, t0, v0, po, oo, x=x1)
    e = rel_err(v1, vo, box)
    print(f"amc {form}: max e = {e.max():.3e}")
    assert e.max() <= 2e-6


@pytest.mark.parametrize("form", ["fp64", "split"])
def test_amc_conserves_angular_momentum_on_gpu(mpc, form):
    """Per cell: sum v and sum r_ic x v unchanged by the GPU's collision (no
    gravity; streaming leaves v unchanged in a periodic box)."""
    L = (24, 24, 24)
    box = box_of(L, seed=3)
    x, v = synth.box_state(L, seed=33)
    t0 = 11
    with mpc.Sim(box, form=form) as sim:
        sim.set_state(x, v)
        x0, v0 = sim.get_state()
        sim.set_step(t0)
        sim.step(1)
        x1, v1 = sim.get_state()
        kg, pg, og = sim.get_binning()
    fr = frame(oparams(box), t0, x1)
    # per-cell sums by bincount over the GPU's keys
    nc = og.size - 1
    rc = np.stack([np.bincount(kg, fr[k], nc) for k in range(3)])
    cnt = np.maximum(np.bincount(kg, minlength=nc), 1)
    r = fr - (rc / cnt)[:, kg]
    sums = {}
    for name, vv in (("before", v0), ("after", v1)):
        Lc = np.cross(r.T, vv.T).T
        sums[name] = (np.stack([np.bincount(kg, vv[k], nc) for k in range(3)]),
                      np.stack([np.bincount(kg, Lc[k], nc) for k in range(3)]))
    tol = 1e-11 if form == "fp64" else 2e-5
    dP = np.abs(sums["after"][0] - sums["before"][0]).max()
    dL = np.abs(sums["after"][1] - sums["before"][1]).max()
    print(f"amc {form}: max per-cell |dP| = {dP:.3e}, |dL| = {dL:.3e}")
    assert dP <= tol * 10 and dL <= tol * 10


def test_amc_with_walls_refused(mpc):
    """No-slip walls would need phantom positions: refused (slip walls are fine)."""
    box = box_of((8, 8, 8), walls=True)
    with pytest.raises(mpc.MPCError) as e:
        mpc.Sim(box)
    assert e.value.code == mpc.EINVAL


def test_amc_thermostat_relaxes_temperature(mpc):
    """SRD+a heats the fluid on its own; with the thermostat the temperature
    relaxes to kT from a hotter start."""
    L = (16, 16, 16)
    with mpc.Sim(box_of(L, seed=4, mbs=True), form="fp64") as sim:
        x, v = synth.box_state(L, seed=44, kT=2.0)
        sim.set_state(x, v)
        sim.step(30)
        T = sim.observables()["T"]
    print(f"amc+mbs: T after 30 steps from kT = 2: {T:.4f}")
    assert abs(T - 1.0) < 0.02


@pytest.mark.parametrize("form,mbs", [("fp64", False), ("fp64", True), ("split", True)])
def test_amc_slip_walls_one_step(mpc, form, mbs):
    """SRD+a next to slip walls (no phantoms), with gravity along x."""
    L = (12, 10, 8)
    box = box_of(L, seed=15, mbs=mbs, walls=True, slip=True, g=(1e-3, 0.0, 0.0))
    x, v = synth.box_state(L, seed=25)
    v *= 2.0
    t0 = 6
    print(f"case amc slip walls form={form} mbs={mbs}", flush=True)
    with mpc.Sim(box, form=form, reorder_every=0) as sim:
        sim.set_state(x, v)
        x0, v0 = sim.get_state()
        sim.set_step(t0)
        sim.step(1)
        x1, v1 = sim.get_state()
        kg, pg, og = sim.get_binning()
    p = orc.Params(L=L, h=box["h"], alpha=box["alpha"], kT=box["kT"], mass=box["mass"],
                   density=box["density"], seed=box["seed"], mbs=mbs, walls=True, slip=True,
                   amc=True, g=box["g"])
    xs, vs, nb = orc.stream(p, x0, v0)
    assert nb > 50
    if form == "fp64":
        np.testing.assert_array_equal(x1, xs)
    ko = orc.keys(p, t0, x1)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    np.testing.assert_array_equal(og, oo)
    vo = orc.collide(p, t0, vs, po, oo, x=x1)
    e = rel_err(v1, vo, box)
    if form == "fp64":
        cond = cell_cond(ko, oo, po, frame(p, t0, x1))
        tol = 1e-12 + 64 * EPS * cond
    else:
        tol = 2e-6
    print(f"amc slip walls {form}: max e = {e.max():.3e}")
    assert np.all(e <= tol)
