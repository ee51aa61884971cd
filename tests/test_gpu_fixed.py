"""GPU tests of the fixed-point cell sums (MPC_FIXED_SUMS, Sec. III.C).

  * Parity with the oracle in the same mode: one step, FP64 e <= 1e-12
    (SRD+a: + 64 eps cond(I_c)), reduced forms e <= 2e-6; positions and
    binning bit-identical.
  * The defining property, on the GPU: the trajectory does not depend on
    the order in which the particles are stored.  After 20 steps from a
    state and from a permutation of it, the states agree bit for bit (and,
    with FP64 sums in the FP64 form, they do not); runs with different
    reorder intervals agree bit for bit as sets of particles.
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


def box_of(L, seed=1, **kw):
    b = dict(L=tuple(L), h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=10.0,
             seed=seed, mbs=False, walls=False, amc=False, fixed=True, g=(0.0, 0.0, 0.0))
    b.update(kw)
    return b


def oparams(box):
    return orc.Params(L=box["L"], h=box["h"], alpha=box["alpha"], kT=box["kT"],
                      mass=box["mass"], density=box["density"], seed=box["seed"],
                      mbs=box["mbs"], walls=box["walls"], amc=box["amc"], fixed=box["fixed"],
                      g=box["g"])


def rel_err(vg, vo, box):
    floor = math.sqrt(box["kT"] / box["mass"])
    return np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), floor)


FIXED_CASES = [
    # L, mbs, walls, amc, gravity, R, t0
    ((16, 16, 16), True, False, False, (0, 0, 0), 0, 0),
    ((13, 9, 11), False, False, False, (0, 0, 0), 1, 3),
    ((12, 10, 8), True, True, False, (2e-3, 0, 0), 3, 2),
    ((12, 10, 8), True, False, True, (0, 0, 0), 0, 4),
    ((10, 10, 10), False, False, True, (0, 0, 0), 1, 6),
]


def test_fixed_batched_boxes(mpc):
    """Fixed-point sums with the thermostat on a batch of uneven boxes (a
    single-cell box among them): each box equals its own oracle step in the
    same mode."""
    shapes = [(10, 7, 9), (1, 1, 1), (6, 11, 4)]
    boxes = [box_of(L, seed=80 + i, mbs=True, kT=0.6 + 0.5 * i) for i, L in enumerate(shapes)]
    states = [synth.box_state(b["L"], density=b["density"], kT=b["kT"], seed=400 + i)
              for i, b in enumerate(boxes)]
    t0 = 2
    with mpc.Sim(boxes, form="fp64", reorder_every=3) as sim:
        for i, (x, v) in enumerate(states):
            sim.set_state(x, v, box=i)
        sim.set_step(t0)
        sim.step(1)
        outs = [sim.get_state(box=i) for i in range(len(boxes))]
        bins = [sim.get_binning(box=i) for i in range(len(boxes))]
    for i, b in enumerate(boxes):
        x, v = states[i]
        xo, vo, ko, po, oo = orc.step(oparams(b), t0, x, v, reorder=True, binning=True)
        np.testing.assert_array_equal(bins[i][0], ko)
        np.testing.assert_array_equal(bins[i][1], po)
        np.testing.assert_array_equal(bins[i][2], oo)
        np.testing.assert_array_equal(outs[i][0], xo)
        e = rel_err(outs[i][1], vo, b)
        print(f"box {i} {b['L']}: max e = {e.max():.3e}")
        assert e.max() <= 1e-12, i


@pytest.mark.parametrize("L,mbs,walls,amc,g,R,t0", FIXED_CASES)
def test_fixed_fp64_one_step(mpc, L, mbs, walls, amc, g, R, t0):
    box = box_of(L, seed=3 + t0, mbs=mbs, walls=walls, amc=amc, g=g)
    x, v = synth.box_state(L, seed=17 + t0)
    print(f"case fixed fp64 L={L} mbs={mbs} walls={walls} amc={amc} R={R} t0={t0}", flush=True)
    with mpc.Sim(box, form="fp64", reorder_every=R) as sim:
        sim.set_state(x, v)
        sim.set_step(t0)
        sim.step(1)
        xg, vg = sim.get_state()
        kg, pg, og = sim.get_binning()
    sorted_out = R > 0 and (t0 + 1) % R == 0
    p = oparams(box)
    xo, vo, ko, po, oo = orc.step(p, t0, x, v, reorder=sorted_out, binning=True)
    np.testing.assert_array_equal(kg, ko)
    np.testing.assert_array_equal(pg, po)
    np.testing.assert_array_equal(og, oo)
    np.testing.assert_array_equal(xg, xo)
    e = rel_err(vg, vo, box)
    tol = 1e-12
    if amc:
        xs, _, _ = orc.stream(p, x, v)
        y = xs + orc.shift(p, t0)[:, None]
        fr = y - np.floor(y)
        cond = np.ones(x.shape[1])
        for c in np.nonzero(np.diff(oo) >= 3)[0]:
            idx = po[oo[c]:oo[c + 1]]
            r = fr[:, idx] - fr[:, idx].mean(axis=1, keepdims=True)
            cond[idx] = np.linalg.cond((r * r).sum() * np.eye(3) - r @ r.T)
        if sorted_out:
            cond = cond[po]
        tol = tol + 64 * EPS * cond
    print(f"fixed fp64: max e = {e.max():.3e}")
    assert np.all(e <= tol)


@pytest.mark.parametrize("form", ["fp32", "split"])
def test_fixed_reduced_precision_one_step(mpc, form):
    L = (16, 12, 10)
    box = box_of(L, seed=9, mbs=True)
    x, v = synth.box_state(L, seed=21)
    t0 = 4
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
    vo = orc.collide(p, t0, v0, po, oo)
    e = rel_err(v1, vo, box)
    print(f"fixed {form}: max e = {e.max():.3e}")
    assert e.max() <= 2e-6


def _run(mpc, box, form, x, v, steps, R=0):
    with mpc.Sim(box, form=form, reorder_every=R) as sim:
        sim.set_state(x, v)
        sim.step(steps)
        return sim.get_state()


@pytest.mark.parametrize("form,mbs,walls,amc", [("fp64", True, False, False),
                                                ("fp64", True, True, False),
                                                ("fp64", True, False, True),
                                                ("split", True, False, False)])
def test_fixed_order_independent(mpc, form, mbs, walls, amc):
    L = (16, 14, 12)
    x, v = synth.box_state(L, seed=61)
    perm = np.random.default_rng(8).permutation(x.shape[1])
    inv = np.argsort(perm)
    same = {}
    for fixed in (False, True):
        box = box_of(L, seed=12, mbs=mbs, walls=walls, amc=amc, fixed=fixed)
        xa, va = _run(mpc, box, form, x, v, 20)
        xb, vb = _run(mpc, box, form, x[:, perm], v[:, perm], 20)
        same[fixed] = bool(np.array_equal(xa, xb[:, inv]) and np.array_equal(va, vb[:, inv]))
    print(f"{form} mbs={mbs} walls={walls} amc={amc}: bitwise equal after 20 steps "
          f"(fp64 sums, fixed sums) = ({same[False]}, {same[True]})")
    assert same[True]
    if form == "fp64":
        # FP64 sums depend on the order at the rounding level; in the split
        # form the FP32 rounding of the cell record usually hides it, without
        # a guarantee
        assert not same[False]


def test_fixed_reorder_interval_independent(mpc):
    """Renumbering the particles (reorder interval R) changes the order of
    every cell's terms; with fixed-point sums the particles' states are the
    same bit for bit (compared as sets, since R renumbers them)."""
    L = (16, 16, 16)
    x, v = synth.box_state(L, seed=71)

    def rows(xs, vs):
        a = np.concatenate([xs, vs]).T
        return a[np.lexsort(a.T[::-1])]

    out = {}
    for fixed in (False, True):
        box = box_of(L, seed=14, mbs=True, fixed=fixed)
        ref = rows(*_run(mpc, box, "fp64", x, v, 15, R=0))
        out[fixed] = [bool(np.array_equal(ref, rows(*_run(mpc, box, "fp64", x, v, 15, R=R))))
                      for R in (1, 4)]
    print(f"R = 1, 4 equal to R = 0: fp64 sums {out[False]}, fixed sums {out[True]}")
    assert all(out[True]) and not any(out[False])


def test_fixed_range_error(mpc):
    """A kinetic-energy summand (formed with the thermostat) of about 2^39."""
    L = (8, 8, 8)
    x, v = synth.box_state(L, seed=5)
    v[:, 3] = [2.0 ** 20, 0.0, 0.0]
    with mpc.Sim(box_of(L, mbs=True), form="fp64") as sim:
        sim.set_state(x, v)
        with pytest.raises(mpc.MPCError) as e:
            sim.step(1)
            sim.sync()
        assert e.value.code == mpc.ERANGE
