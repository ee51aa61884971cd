"""GPU tests of the wall variants (Sec. II, Boundary conditions): slip walls
(specular reflection, no phantoms) and no-slip walls moving along x (shear
flow between walls at +-U).

  * One step against the oracle: FP64 positions and binning bit-identical,
    velocities e <= 1e-12; FP32 and split forms as in the other parity tests
    (binning given the GPU's post-stream state, collision e <= 2e-6).
  * Physics on the GPU: slip walls exert no tangential force (momentum grows
    by N m g h per step to rounding); moving walls give the linear Couette
    profile with slope 2U/H.
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


def box_of(L, seed=1, slip=False, uwall=0.0, mbs=True, g=(0.0, 0.0, 0.0), **kw):
    b = dict(L=tuple(L), h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=10.0,
             seed=seed, mbs=mbs, walls=True, slip=slip, uwall=uwall, g=tuple(g))
    b.update(kw)
    return b


def oparams(box):
    return orc.Params(L=box["L"], h=box["h"], alpha=box["alpha"], kT=box["kT"],
                      mass=box["mass"], density=box["density"], seed=box["seed"],
                      mbs=box["mbs"], walls=True, slip=box["slip"], uwall=box["uwall"],
                      g=box["g"])


def rel_err(vg, vo, box):
    floor = math.sqrt(box["kT"] / box["mass"])
    return np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), floor)


WALL_CASES = [
    # L, slip, U, mbs, gravity, R, t0
    ((12, 10, 8), True, 0.0, True, (2e-3, 0, 0), 0, 2),
    ((13, 9, 11), True, 0.0, False, (0, 0, 0), 1, 5),
    ((12, 10, 8), False, 0.3, True, (0, 0, 0), 0, 3),
    ((13, 9, 7), False, 0.5, True, (1e-3, 0, 0), 1, 8),
    ((16, 16, 6), False, 0.2, False, (0, 0, 0), 3, 2),
    ((3, 2, 2), True, 0.0, True, (1e-3, 0, 0), 0, 2),     # slip walls, H = 2
    ((2, 2, 1), False, 0.3, True, (0, 0, 0), 1, 1),       # moving walls, H = 1
]


@pytest.mark.parametrize("L,slip,U,mbs,g,R,t0", WALL_CASES)
def test_walls_fp64_one_step(mpc, L, slip, U, mbs, g, R, t0):
    box = box_of(L, seed=5 + t0, slip=slip, uwall=U, mbs=mbs, g=g)
    x, v = synth.box_state(L, seed=31 + t0)
    v *= 2.0  # more wall crossings
    print(f"case walls fp64 L={L} slip={slip} U={U} mbs={mbs} R={R} t0={t0}", flush=True)
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
    print(f"walls fp64: max e = {e.max():.3e}")
    assert e.max() <= 1e-12


@pytest.mark.parametrize("form,slip,U", [("fp32", True, 0.0), ("split", True, 0.0),
                                         ("fp32", False, 0.4), ("split", False, 0.4)])
def test_walls_reduced_precision_one_step(mpc, form, slip, U):
    L = (16, 12, 10)
    box = box_of(L, seed=9, slip=slip, uwall=U)
    x, v = synth.box_state(L, seed=23)
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
    xs, vs, nb = orc.stream(p, x0, v0)
    assert nb > 100
    dx = np.abs(x1 - xs)
    for k in range(2):
        dx[k] = np.minimum(dx[k], L[k] - dx[k])
    print(f"walls {form}: max stream error {dx.max():.3e} cells, {nb} crossings")
    assert dx.max() < (2e-4 if form == "fp32" else 2e-6)
    ko = orc.keys(p, t0, x1)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    np.testing.assert_array_equal(og, oo)
    vo = orc.collide(p, t0, vs, po, oo)
    e = rel_err(v1, vo, box)
    print(f"walls {form}: max e = {e.max():.3e}")
    assert e.max() <= 2e-6


def test_slip_walls_no_tangential_force(mpc):
    L = (32, 32, 16)
    g = 1e-3
    box = box_of(L, seed=4, slip=True, g=(g, 0.0, 0.0))
    x, v = synth.box_state(L, seed=41)
    n = x.shape[1]
    with mpc.Sim(box, form="fp64") as sim:
        sim.set_state(x, v)
        p0 = sim.observables()["P"]
        sim.step(200)
        p1 = sim.observables()["P"]
    expect = n * g * 0.1 * 200
    print(f"slip walls: dP_x = {p1[0] - p0[0]:.9f}, N m g h steps = {expect:.9f}")
    assert abs((p1[0] - p0[0]) - expect) < 1e-9 * n
    assert abs(p1[1] - p0[1]) < 1e-9 * n


def test_couette_profile_gpu(mpc):
    """Walls at +-U: time-averaged v_x(z) linear, slope within 5 % of 2U/H
    (the small slip at the walls lowers it by a few per cent)."""
    L = (32, 32, 16)
    U = 0.4
    box = box_of(L, seed=6, uwall=U)
    nb = 32
    acc = np.zeros(nb)
    cnt = np.zeros(nb)
    with mpc.Sim(box, form="fp64") as sim:
        sim.init_state(5)
        sim.step(1500)
        for _ in range(60):
            sim.step(25)
            x, v = sim.get_state()
            b = np.minimum((x[2] / L[2] * nb).astype(int), nb - 1)
            acc += np.bincount(b, v[0], nb)
            cnt += np.bincount(b, minlength=nb)
    z = (np.arange(nb) + 0.5) * L[2] / nb
    prof = acc / cnt
    slope, icpt = np.polyfit(z - L[2] / 2, prof, 1)
    resid = prof - (slope * (z - L[2] / 2) + icpt)
    r2 = 1 - (resid ** 2).sum() / ((prof - prof.mean()) ** 2).sum()
    print(f"Couette GPU: slope/theory {slope / (2 * U / L[2]):.4f}, intercept {icpt:.4f}, "
          f"R2 {r2:.5f}")
    assert abs(slope / (2 * U / L[2]) - 1) < 0.05
    assert abs(icpt) < 0.01 and r2 > 0.995


def test_wall_flag_validation(mpc):
    with pytest.raises(mpc.MPCError) as e:
        mpc.Sim(dict(box_of((8, 8, 8)), walls=False, slip=True))
    assert e.value.code == mpc.EINVAL
    with pytest.raises(mpc.MPCError) as e:
        mpc.Sim(box_of((8, 8, 8), slip=True, uwall=0.1))
    assert e.value.code == mpc.EINVAL


@pytest.mark.parametrize("kw", [dict(slip=True, g=(2e-3, 0.0, 0.0)), dict(uwall=0.3),
                                dict(uwall=0.3, fixed=True)])
def test_walls_20_steps_graph(mpc, kw):
    """20 steps replayed from a captured graph against the oracle run."""
    L = (12, 10, 8)
    box = box_of(L, seed=10, **kw)
    x, v = synth.box_state(L, seed=83)
    with mpc.Sim(box, form="fp64", graph=True) as sim:
        sim.set_state(x, v)
        sim.step(20)
        xg, vg = sim.get_state()
    p = oparams(box)
    p.fixed = bool(kw.get("fixed", False))
    xo, vo = orc.run(p, x, v, 20)
    d = np.abs(xg - xo)
    for k in range(2):
        d[k] = np.minimum(d[k], L[k] - d[k])
    e = rel_err(vg, vo, box)
    print(f"walls {kw} 20 steps: max |dx| = {d.max():.3e}, max e = {e.max():.3e}")
    assert d.max() < 1e-10 and e.max() < 1e-10
