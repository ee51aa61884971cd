"""GPU tests of the Lees-Edwards shear of a periodic box (Sec. II, boundary
conditions; mpc_params.le_u).

  * One step against the oracle: FP64 positions and binning bit-identical,
    velocities e <= 1e-12 (with the thermostat, fixed-point sums, gravity and
    several reorder intervals); FP32 and split forms with the usual bars.
  * Momentum budget on the GPU: a step changes the total x momentum only by
    U (n_down - n_up), the face crossings.
  * The steady shear profile: v_x(z) linear with slope U / L_z.
  * SRD+a under the shear against the oracle (image positions and velocities
    in the cells across the z faces).
"""
import math

import numpy as np
import pytest

import oracle as orc
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


def box_of(L, U, seed=1, mbs=True, fixed=False, g=(0.0, 0.0, 0.0), **kw):
    b = dict(L=tuple(L), h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=10.0,
             seed=seed, mbs=mbs, walls=False, fixed=fixed, le_u=U, g=tuple(g))
    b.update(kw)
    return b


def oparams(box):
    return orc.Params(L=box["L"], h=box["h"], alpha=box["alpha"], kT=box["kT"],
                      mass=box["mass"], density=box["density"], seed=box["seed"],
                      mbs=box["mbs"], fixed=box["fixed"], le_u=box["le_u"], g=box["g"])


def rel_err(vg, vo, box):
    floor = math.sqrt(box["kT"] / box["mass"])
    return np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), floor)


LE_CASES = [
    # L, U, mbs, fixed, gravity, R, t0
    ((16, 16, 16), 0.5, True, False, (0, 0, 0), 0, 0),
    ((13, 9, 11), 0.8, False, False, (0, 0, 0), 1, 3),
    ((12, 10, 8), 0.3, True, True, (1e-3, 0, 0), 3, 2),
    ((7, 33, 5), 1.7, True, False, (0, 0, 0), 0, 123456),
    ((4, 3, 2), 0.7, True, False, (0, 0, 0), 1, 4),      # two layers across the shear
    ((3, 2, 1), 0.4, False, False, (0, 0, 0), 0, 2),     # one layer: its own image
]


@pytest.mark.parametrize("L,U,mbs,fixed,g,R,t0", LE_CASES)
def test_lees_edwards_fp64_one_step(mpc, L, U, mbs, fixed, g, R, t0):
    box = box_of(L, U, seed=5 + t0 % 97, mbs=mbs, fixed=fixed, g=g)
    x, v = synth.box_state(L, seed=37 + t0 % 89)
    v *= 2.0  # more face crossings
    print(f"case le fp64 L={L} U={U} mbs={mbs} fixed={fixed} R={R} t0={t0}", flush=True)
    with mpc.Sim(box, form="fp64", reorder_every=R) as sim:
        sim.set_state(x, v)
        sim.set_step(t0)
        sim.step(1)
        xg, vg = sim.get_state()
        kg, pg, og = sim.get_binning()
    sorted_out = R > 0 and (t0 + 1) % R == 0
    xo, vo, ko, po, oo = orc.step(oparams(box), t0, x, v, reorder=sorted_out, binning=True)
    np.testing.assert_array_equal(kg, ko)
    np.testing.assert_array_equal(pg, po)
    np.testing.assert_array_equal(og, oo)
    np.testing.assert_array_equal(xg, xo)
    e = rel_err(vg, vo, box)
    print(f"le fp64: max e = {e.max():.3e}")
    assert e.max() <= 1e-12


@pytest.mark.parametrize("form", ["fp32", "split"])
def test_lees_edwards_reduced_precision_one_step(mpc, form):
    L = (16, 12, 10)
    U = 0.6
    box = box_of(L, U, seed=9)
    x, v = synth.box_state(L, seed=27)
    v *= 2.0
    t0 = 4
    with mpc.Sim(box, form=form) as sim:
        sim.set_state(x, v)
        x0, v0 = sim.get_state()
        sim.set_step(t0)
        sim.step(1)
        x1, v1 = sim.get_state()
        kg, pg, og = sim.get_binning()
    p = oparams(box)
    xs, vs, _ = orc.stream(p, x0, v0, t=t0)
    dx = np.abs(x1 - xs)
    for k in range(3):
        dx[k] = np.minimum(dx[k], L[k] - dx[k])
    print(f"le {form}: max stream error {dx.max():.3e} cells")
    assert dx.max() < 2e-5
    ko = orc.keys(p, t0, x1)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    np.testing.assert_array_equal(og, oo)
    np.testing.assert_array_equal(pg, po)
    vo = orc.collide(p, t0, vs, po, oo, x=x1)
    e = rel_err(v1, vo, box)
    print(f"le {form}: max e = {e.max():.3e}")
    assert e.max() <= 2e-6


def test_lees_edwards_momentum_budget_gpu(mpc):
    L = (32, 32, 16)
    U, t0 = 0.7, 5
    box = box_of(L, U, seed=4)
    x, v = synth.box_state(L, seed=43)
    v *= 2.0
    zend = x[2] + 0.1 * v[2]
    n_up, n_down = int((zend >= L[2]).sum()), int((zend < 0).sum())
    with mpc.Sim(box, form="fp64") as sim:
        sim.set_state(x, v)
        sim.set_step(t0)
        p0 = sim.observables()["P"]
        sim.step(1)
        p1 = sim.observables()["P"]
    print(f"le budget: dP_x = {p1[0] - p0[0]:.9f}, U (n_down - n_up) = {U * (n_down - n_up):.9f}")
    assert abs((p1[0] - p0[0]) - U * (n_down - n_up)) < 1e-10 * x.shape[1]


def test_lees_edwards_shear_profile_gpu(mpc):
    L = (32, 32, 24)
    U = 0.6
    box = box_of(L, U, seed=6)
    nb = 24
    acc = np.zeros(nb)
    cnt = np.zeros(nb)
    with mpc.Sim(box, form="fp64") as sim:
        sim.init_state(3)
        sim.step(1500)
        for _ in range(60):
            sim.step(25)
            x, v = sim.get_state()
            b = np.minimum((x[2] / L[2] * nb).astype(int), nb - 1)
            acc += np.bincount(b, v[0], nb)
            cnt += np.bincount(b, minlength=nb)
    z = (np.arange(nb) + 0.5) * L[2] / nb
    prof = acc / cnt
    slope, icpt = np.polyfit(z, prof, 1)
    resid = prof - (slope * z + icpt)
    r2 = 1 - (resid ** 2).sum() / ((prof - prof.mean()) ** 2).sum()
    print(f"Lees-Edwards GPU: slope/theory {slope / (U / L[2]):.4f}, R2 {r2:.5f}")
    assert abs(slope / (U / L[2]) - 1) < 0.03 and r2 > 0.995


def test_lees_edwards_flag_validation(mpc):
    with pytest.raises(mpc.MPCError) as e:
        mpc.Sim(box_of((8, 8, 8), 0.3, walls=True))
    assert e.value.code == mpc.EINVAL


EPS = 2.0 ** -52


@pytest.mark.parametrize("form,mbs", [("fp64", False), ("fp64", True), ("split", True)])
def test_lees_edwards_with_amc_one_step(mpc, form, mbs):
    """SRD+a under Lees-Edwards shear: image positions and velocities in the
    cells across the z faces.  FP64 e <= 1e-12 + 64 eps cond(I_c)."""
    L = (12, 10, 8)
    U, t0 = 0.7, 9
    box = box_of(L, U, seed=17, mbs=mbs, amc=True)
    x, v = synth.box_state(L, seed=29)
    v *= 2.0
    print(f"case le amc form={form} mbs={mbs}", flush=True)
    with mpc.Sim(box, form=form) as sim:
        sim.set_state(x, v)
        x0, v0 = sim.get_state()
        sim.set_step(t0)
        sim.step(1)
        x1, v1 = sim.get_state()
        kg, pg, og = sim.get_binning()
    p = orc.Params(L=L, h=box["h"], alpha=box["alpha"], kT=box["kT"], mass=box["mass"],
                   density=box["density"], seed=box["seed"], mbs=mbs, amc=True, le_u=U)
    xs, vs, _ = orc.stream(p, x0, v0, t=t0)
    if form == "fp64":
        np.testing.assert_array_equal(x1, xs)
    ko = orc.keys(p, t0, x1)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    vo = orc.collide(p, t0, vs, po, oo, x=x1)
    e = rel_err(v1, vo, box)
    tol = 2e-6
    if form == "fp64":
        s = orc.shift(p, t0)
        d = (U * (t0 + 1) * box["h"]) % L[0]
        cz = np.floor(x1[2] + s[2])
        side = np.where(cz < 0, 1.0, np.where(cz >= L[2], -1.0, 0.0))
        xm = x1.copy()
        xm[0] += side * d
        y = xm + s[:, None]
        fr = y - np.floor(y)
        cond = np.ones(x1.shape[1])
        for c in np.nonzero(np.diff(oo) >= 3)[0]:
            idx = po[oo[c]:oo[c + 1]]
            r = fr[:, idx] - fr[:, idx].mean(axis=1, keepdims=True)
            cond[idx] = np.linalg.cond((r * r).sum() * np.eye(3) - r @ r.T)
        tol = 1e-12 + 64 * EPS * cond
    print(f"le amc {form}: max e = {e.max():.3e}")
    assert np.all(e <= tol)


@pytest.mark.parametrize("kind", ["lees_edwards", "moving_walls"])
def test_batched_boxes_with_different_boundary_velocities(mpc, kind):
    """One handle, boxes with different le_u (some 0) or different wall
    velocities: each box equals its own oracle step (the sheared kernel runs
    the unsheared boxes with the per-box flag off)."""
    if kind == "lees_edwards":
        boxes = [box_of((10, 8, 9), 0.5, seed=3), box_of((7, 9, 6), 0.0, seed=4),
                 box_of((12, 6, 8), -0.3, seed=5)]
    else:
        boxes = [dict(box_of((10, 8, 9), 0.0, seed=3), walls=True, uwall=0.2),
                 dict(box_of((7, 9, 6), 0.0, seed=4), walls=True, uwall=0.0),
                 dict(box_of((12, 6, 8), 0.0, seed=5), walls=True, uwall=-0.4)]
    states = []
    for i, b in enumerate(boxes):
        x, v = synth.box_state(b["L"], seed=50 + i)
        states.append((x, 2.0 * v))
    t0 = 7
    with mpc.Sim(boxes, form="fp64", reorder_every=0) as sim:
        for i, (x, v) in enumerate(states):
            sim.set_state(x, v, box=i)
        sim.set_step(t0)
        sim.step(1)
        outs = [sim.get_state(box=i) for i in range(len(boxes))]
        bins = [sim.get_binning(box=i) for i in range(len(boxes))]
    for i, b in enumerate(boxes):
        x, v = states[i]
        p = orc.Params(L=b["L"], h=b["h"], alpha=b["alpha"], kT=b["kT"], mass=b["mass"],
                       density=b["density"], seed=b["seed"], mbs=b["mbs"], walls=b["walls"],
                       le_u=b["le_u"], uwall=b.get("uwall", 0.0), g=b["g"])
        xo, vo, ko, po, oo = orc.step(p, t0, x, v, binning=True)
        np.testing.assert_array_equal(bins[i][0], ko)
        np.testing.assert_array_equal(bins[i][1], po)
        np.testing.assert_array_equal(bins[i][2], oo)
        np.testing.assert_array_equal(outs[i][0], xo)
        e = rel_err(outs[i][1], vo, b)
        print(f"{kind} box {i}: max e = {e.max():.3e}")
        assert e.max() <= 1e-12, (i, e.max())


def test_lees_edwards_20_steps_graph(mpc):
    """20 steps replayed from a captured graph (the offset d(t) advances every
    step) against the oracle run from the same state."""
    L = (16, 16, 16)
    U = 0.8
    box = box_of(L, U, seed=8)
    x, v = synth.box_state(L, seed=81)
    with mpc.Sim(box, form="fp64", graph=True) as sim:
        sim.set_state(x, v)
        sim.step(20)
        xg, vg = sim.get_state()
    xo, vo = orc.run(oparams(box), x, v, 20)
    d = np.abs(xg - xo)
    d = np.minimum(d, 16.0 - d)
    e = rel_err(vg, vo, box)
    print(f"le 20 steps: max |dx| = {d.max():.3e}, max e = {e.max():.3e}")
    assert d.max() < 1e-10 and e.max() < 1e-10
