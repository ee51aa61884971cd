"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against what the paper (arXiv:2406.15236) and
the mathematics fix: an independent library routine, exact rational
arithmetic, a closed form, a conservation law or a distribution.  None of
them re-types the oracle's own formula.
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.transform import Rotation

import synth

DEG = math.pi / 180.0


# --------------------------------------------------------------------------
# Random streams
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND reference")
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand.cpp")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_philox):
    """Philox4x32-10 block function equals rocRAND's independent implementation."""
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2**32, size=(4000, 6), dtype=np.uint64)
    rows[:8] = [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6, [0, 0, 0, 0, 2**32 - 1, 0],
                [1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0],
                [0, 0, 0, 1, 0, 0], [5, 17, 100, 3, 1, 0]]
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        ref = [int(v) for v in line.split()]
        got = orc.philox(r[:4], r[4:])
        assert list(got) == ref, (r, got, ref)


def test_uniform_conversions(orc):
    """Range, grid and end points of the word -> uniform conversions."""
    assert orc.u24(0) == 0.0 and orc.u24(0xFFFFFFFF) == 1.0 - 2.0**-24
    assert orc.u24(0xFF) == 0.0 and orc.u24(0x100) == 2.0**-24
    assert orc.u53(0, 0) == 0.0 and orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert orc.u53(0, 1 << 11) == 2.0**-53 and orc.u53(1, 0) == 2.0**-32
    lo, hi = orc.u53_open(0, 0), orc.u53_open(0xFFFFFFFF, 0xFFFFFFFF)
    assert 0.0 < lo and hi < 1.0 and lo + hi == 1.0
    assert 0.0 < orc.u32_open(0) and orc.u32_open(0xFFFFFFFF) < 1.0
    assert orc.u32_open(0) + orc.u32_open(0xFFFFFFFF) == 1.0
    rng = np.random.default_rng(3)
    for a, b in rng.integers(0, 2**32, size=(200, 2)):
        u = orc.u53(int(a), int(b))
        assert 0.0 <= u < 1.0 and Fraction(u) * 2**53 == int(Fraction(u) * 2**53)


def test_shift_grid_and_uniformity(orc):
    """Sec. II: one random lattice shift per step, uniform in [-a/2, a/2)^3."""
    p = orc.Params(seed=11)
    s = np.array([orc.shift(p, t) for t in range(4000)])
    assert s.min() >= -0.5 and s.max() < 0.5
    assert np.all(s * 2**24 == np.round(s * 2**24))  # exact 2^-24 grid
    for k in range(3):
        assert stats.kstest(s[:, k], stats.uniform(-0.5, 1.0).cdf).pvalue > 1e-3
    assert abs(np.corrcoef(s[:-1, 0], s[1:, 0])[0, 1]) < 0.06
    assert not np.array_equal(orc.shift(p, 5), orc.shift(orc.Params(seed=12), 5))


# --------------------------------------------------------------------------
# Streaming, Eq.(1)
# --------------------------------------------------------------------------
def _wrapped_exact(x, h, v, L):
    """x + h v in exact rational arithmetic, then brought into [0, L)."""
    e = Fraction(x) + Fraction(h) * Fraction(v)
    while e < 0:
        e += L
    while e >= L:
        e -= L
    return e


def test_stream_exact_single_rounding(orc):
    """Eq.(1): r <- r + h v with one rounding (fma) and periodic images."""
    L = (16, 8, 12)
    p = orc.Params(L=L, h=0.1)
    x, v = synth.box_state(L, n=3000, seed=5)
    v[:, :50] *= 30.0  # some particles cross the boundary
    x2, v2, nb = orc.stream(p, x, v)
    assert nb == 0 and np.array_equal(v2, v)
    for k in range(3):
        for i in range(x.shape[1]):
            ex = _wrapped_exact(x[k, i], p.h, v[k, i], L[k])
            e_unwrapped = Fraction(x[k, i]) + Fraction(p.h) * Fraction(v[k, i])
            got = Fraction(x2[k, i])
            assert 0 <= x2[k, i] < L[k]
            xe = float(e_unwrapped)  # one correctly rounded x + h v
            if 0 <= xe < L[k]:
                assert x2[k, i] == xe
            else:
                # one periodic image, itself correctly rounded (wrap reading)
                img = float(Fraction(xe) + (L[k] if xe < 0 else -L[k]))
                img = 0.0 if img == L[k] else img
                assert x2[k, i] == img
                d = abs(got - ex)
                assert min(d, L[k] - d) <= Fraction(2.0**-50) * L[k]


def test_stream_wraps_far_outside(orc):
    """Displacements of many box lengths in one step (Eq. (1) with periodic
    images): the stored position is the once-rounded x + h v taken modulo L,
    in [0, L), to a few ulps of L."""
    L = (3, 2, 5)
    p = orc.Params(L=L, h=1.0)
    rng = np.random.default_rng(9)
    n = 4000
    x = np.stack([rng.random(n) * L[k] for k in range(3)])
    v = rng.uniform(-40.0, 40.0, size=(3, n))
    x2, v2, nb = orc.stream(p, x, v)
    assert nb == 0 and np.array_equal(v2, v)
    for k in range(3):
        assert np.all((x2[k] >= 0.0) & (x2[k] < L[k]))
        for i in range(n):
            xe = Fraction(float(Fraction(x[k, i]) + Fraction(v[k, i])))  # one rounding
            ex = xe - L[k] * math.floor(xe / L[k])
            d = abs(Fraction(x2[k, i]) - ex)
            assert min(d, L[k] - d) <= Fraction(2.0**-48) * L[k], (k, i)


def test_stream_wrap_corner(orc):
    """A particle landing a hair below 0 maps into [0, L), never onto L."""
    p = orc.Params(L=(4, 4, 4), h=1.0)
    x = np.array([[1e-18, 3.5, 0.0], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    v = np.array([[-2e-18, 0.5, -0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    x2, _, _ = orc.stream(p, x, v)
    assert np.all(x2 >= 0) and np.all(x2 < 4)
    assert x2[0, 0] == 0.0          # 4 - 1e-18 rounds to 4 -> corner rule gives 0
    assert x2[0, 1] == 0.0          # 3.5 + 0.5 == L exactly -> 0


def test_bounce_back_walls(orc):
    """No-slip walls: particles crossing z=0 or z=H are mirrored back onto the
    fluid side with all velocity components reversed; time reversal restores
    the start (Sec. II, Boundary conditions)."""
    L = (8, 8, 6)
    p = orc.Params(L=L, h=0.5, walls=True)
    x, v = synth.box_state(L, n=5000, seed=9)
    v *= 3.0
    x2, v2, nb = orc.stream(p, x, v)
    zend = x[2] + p.h * v[2]
    crossed = (zend < 0) | (zend > L[2])
    assert nb == int(crossed.sum()) > 100
    assert np.all((x2[2] >= 0) & (x2[2] <= L[2]))
    assert np.array_equal(v2[:, crossed], -v[:, crossed])
    assert np.array_equal(v2[:, ~crossed], v[:, ~crossed])
    bot = crossed & (zend < 0)
    top = crossed & (zend > L[2])
    np.testing.assert_allclose(x2[2, bot], -zend[bot], atol=1e-13)
    np.testing.assert_allclose(x2[2, top], 2 * L[2] - zend[top], atol=1e-13)
    # x, y: the particle travels the reflected path, r_end - 2 v t_rem
    trem = np.where(bot, zend / v[2], (zend - L[2]) / v[2])
    for k in range(2):
        exp = (x[k] + p.h * v[k] - 2 * v[k] * trem) % L[k]
        d = np.abs(x2[k, crossed] - exp[crossed])
        assert np.all(np.minimum(d, L[k] - d) < 1e-12)
    # time reversal: stream back with reversed velocities
    x3, v3, _ = orc.stream(p, x2, -v2)
    for k in range(3):
        d = np.abs(x3[k] - x[k])
        if k < 2:
            d = np.minimum(d, L[k] - d)
        assert d.max() < 1e-12
    np.testing.assert_array_equal(-v3, v)


# --------------------------------------------------------------------------
# Binning
# --------------------------------------------------------------------------
def _exact_key(xi, s, L, walls):
    c = [math.floor(Fraction(float(xi[k])) + Fraction(float(s[k]))) for k in range(3)]
    c[0] %= L[0]
    c[1] %= L[1]
    if walls:
        c[2] += 1
        dims = (L[2] + 2, L[1], L[0])
    else:
        c[2] %= L[2]
        dims = (L[2], L[1], L[0])
    return int(np.ravel_multi_index((c[2], c[1], c[0]), dims))


@pytest.mark.parametrize("walls", [False, True])
def test_keys_exact_floor(orc, walls):
    """key = linear index (x fastest) of floor(x + s) mod L, by exact arithmetic,
    including particles placed exactly on shifted cell faces."""
    L = (7, 5, 6)
    p = orc.Params(L=L, walls=walls, seed=21)
    rng = np.random.default_rng(2)
    for t in range(6):
        s = orc.shift(p, t)
        x, _ = synth.box_state(L, n=800, seed=100 + t)
        # faces: x = j - s (exactly representable), and the box ends
        for k in range(3):
            j = rng.integers(0, L[k] + 1, size=60)
            face = j.astype(float) - s[k]
            ok = (face >= 0) & (face < L[k])
            x[k, :60] = np.where(ok, face, x[k, :60])
        x[:, 60] = 0.0
        x[:, 61] = [np.nextafter(L[0], 0), np.nextafter(L[1], 0), np.nextafter(L[2], 0)]
        key = orc.keys(p, t, x)
        ref = [_exact_key(x[:, i], s, L, walls) for i in range(x.shape[1])]
        assert list(key) == ref


def test_counting_sort_matches_numpy(orc):
    """Stable counting sort == numpy stable argsort, offsets == cumsum(bincount)."""
    rng = np.random.default_rng(4)
    for ncell, n in [(1, 0), (1, 7), (64, 1000), (4096, 40960), (1000, 3)]:
        key = rng.integers(0, ncell, size=n).astype(np.uint32)
        perm, off = orc.sort(key, ncell)
        np.testing.assert_array_equal(perm, np.argsort(key, kind="stable"))
        ref = np.concatenate([[0], np.cumsum(np.bincount(key, minlength=ncell))])
        np.testing.assert_array_equal(off, ref)


# --------------------------------------------------------------------------
# Collision, Eq.(2), and the MBS thermostat
# --------------------------------------------------------------------------
def _one_step_parts(orc, p, t, x, v):
    xs, vs, _ = orc.stream(p, x, v)
    key = orc.keys(p, t, xs)
    perm, off = orc.sort(key, p.ncells)
    v2, cells = orc.collide(p, t, vs, perm, off, cells=True)
    return xs, vs, key, perm, off, v2, cells


def test_rotation_matches_scipy(orc):
    """Rodrigues rotation == scipy Rotation.from_rotvec(alpha n).apply(u)."""
    rng = np.random.default_rng(8)
    for _ in range(500):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        u = rng.normal(size=3)
        a = rng.uniform(0, 2 * math.pi)
        ref = Rotation.from_rotvec(a * n).apply(u)
        np.testing.assert_allclose(orc.rotate(a, n, u), ref, rtol=0, atol=1e-14)
    n = np.array([0.0, 0.0, 1.0])
    np.testing.assert_allclose(orc.rotate(math.pi / 2, n, [1.0, 0, 0]), [0, 1, 0], atol=1e-16)


def test_cell_sums_against_fsum(orc):
    """Cell mean velocity and relative kinetic term vs correctly rounded sums."""
    L = (6, 6, 6)
    p = orc.Params(L=L, mbs=True, seed=3)
    x, v = synth.box_state(L, seed=31)
    xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, 0, x, v)
    for c in range(p.ncells):
        idx = np.nonzero(key == c)[0]
        if idx.size == 0:
            continue
        assert cells[c, 0] == idx.size
        Vex = [math.fsum(vs[k, idx]) / idx.size for k in range(3)]
        np.testing.assert_allclose(cells[c, 2:5], Vex, rtol=0, atol=4e-16 * max(1, idx.size))
        Kex = math.fsum(((vs[:, idx] - np.array(Vex)[:, None]) ** 2).ravel())
        assert abs(cells[c, 5] - Kex) <= 1e-13 * max(Kex, 1e-300) + 1e-15


@pytest.mark.parametrize("mbs", [False, True])
def test_collision_is_rotation_of_relative_velocity(orc, mbs):
    """Eq.(2): v' - v_cm = kappa * R(alpha, n)(v - v_cm) per particle, with R from
    scipy and the cell's axis; kappa = 1 without the thermostat."""
    L = (5, 6, 4)
    p = orc.Params(L=L, mbs=mbs, seed=17, alpha=1.9)
    x, v = synth.box_state(L, seed=41)
    xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, 3, x, v)
    for c in range(p.ncells):
        idx = np.nonzero(key == c)[0]
        if idx.size < 2:
            np.testing.assert_array_equal(v2[:, idx], vs[:, idx])  # unchanged
            continue
        V = cells[c, 2:5]
        n = cells[c, 6:9]
        assert abs(np.linalg.norm(n) - 1) < 1e-15
        kappa = cells[c, 9]
        if not mbs:
            assert kappa == 1.0
        R = Rotation.from_rotvec(p.alpha * n)
        ref = V[:, None] + kappa * R.apply((vs[:, idx] - V[:, None]).T).T
        np.testing.assert_allclose(v2[:, idx], ref, rtol=0, atol=1e-14)


def test_per_cell_momentum_and_energy_conservation(orc):
    """Sec. II: the collision conserves momentum per cell, and without the
    thermostat also kinetic energy per cell."""
    L = (8, 8, 8)
    p = orc.Params(L=L, seed=5)
    x, v = synth.box_state(L, seed=51)
    xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, 7, x, v)
    for c in range(p.ncells):
        idx = np.nonzero(key == c)[0]
        if idx.size == 0:
            continue
        scale = np.abs(vs[:, idx]).sum()
        dP = np.abs(v2[:, idx].sum(axis=1) - vs[:, idx].sum(axis=1)).max()
        assert dP <= 8 * 2.2e-16 * scale * max(1, idx.size)
        E0, E1 = (vs[:, idx] ** 2).sum(), (v2[:, idx] ** 2).sum()
        assert abs(E1 - E0) <= 1e-14 * E0 + 1e-300


def test_special_angles(orc):
    """alpha = 0 leaves v unchanged; alpha = pi gives u' = 2 (n.u) n - u."""
    L = (4, 4, 4)
    x, v = synth.box_state(L, seed=61)
    for alpha in (0.0, math.pi):
        p = orc.Params(L=L, alpha=alpha, seed=2)
        xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, 1, x, v)
        for c in range(p.ncells):
            idx = np.nonzero(key == c)[0]
            if idx.size < 2:
                continue
            V, n = cells[c, 2:5], cells[c, 6:9]
            u = vs[:, idx] - V[:, None]
            ref = u if alpha == 0.0 else 2 * (n @ u) * n[:, None] - u
            np.testing.assert_allclose(v2[:, idx] - V[:, None], ref, atol=2e-15)


def test_axis_uniform_on_sphere(orc):
    """Sec. II: the rotation axis is random and independent per cell and step."""
    p = orc.Params(seed=9)
    n = np.array([orc.cell_axis(p, t, c) for t in range(5) for c in range(1200)])
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, atol=2e-16)
    assert stats.kstest(n[:, 2], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    phi = np.arctan2(n[:, 1], n[:, 0])
    assert stats.kstest(phi, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 1e-3
    assert np.abs(n.mean(axis=0)).max() < 0.05
    assert not np.allclose(orc.cell_axis(p, 0, 3), orc.cell_axis(p, 1, 3))


@pytest.mark.parametrize("shape", [1.5, 3.0, 13.5, 28.5])
def test_gamma_sampler_distribution(orc, shape):
    """Sec. II (Thermostat): E_k ~ Gamma(f/2, kT); Marsaglia-Tsang sampler vs scipy."""
    p = orc.Params(seed=77)
    g = np.empty(6000)
    att = np.empty(6000, dtype=int)
    for i in range(g.size):
        g[i], att[i] = orc.cell_gamma(p, i // 1000, i % 1000, shape)
    assert att.min() >= 1 and att.mean() < 1.2
    assert stats.kstest(g, stats.gamma(shape).cdf).pvalue > 1e-3
    assert abs(g.mean() / shape - 1) < 4 * math.sqrt(1 / (shape * g.size)) + 1e-3


def test_mbs_sets_cell_energy_to_drawn_value(orc):
    """MBS: after the collision the relative kinetic energy of each cell equals
    the drawn E_k, whose law is Gamma(3(N_c-1)/2, kT)."""
    L = (10, 10, 10)
    p = orc.Params(L=L, mbs=True, kT=1.7, seed=13)
    x, v = synth.box_state(L, seed=71, kT=0.6)
    xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, 2, x, v)
    sel = cells[:, 0] >= 2
    Ek, Kpost = cells[sel, 10], cells[sel, 15]
    np.testing.assert_allclose(Kpost, 2 * Ek, rtol=1e-12)
    n = cells[sel, 0]
    z = Ek / p.kT
    shape = 1.5 * (n - 1)
    u = stats.gamma.cdf(z, shape)  # probability integral transform
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_mbs_thermalises(orc):
    """With MBS the temperature relaxes to kT from a hotter start."""
    L = (8, 8, 8)
    p = orc.Params(L=L, mbs=True, kT=1.0, seed=23)
    x, v = synth.box_state(L, kT=2.5, seed=81)
    x, v = orc.run(p, x, v, 20)
    T = orc.observables(p, v)["T"]
    assert abs(T - 1.0) < 0.03


def test_storage_order_invariance(orc):
    """The step does not depend on how particles are stored."""
    L = (6, 5, 7)
    p = orc.Params(L=L, mbs=True, seed=29)
    x, v = synth.box_state(L, seed=91)
    q = np.random.default_rng(0).permutation(x.shape[1])
    xa, va = orc.step(p, 4, x, v)
    xb, vb = orc.step(p, 4, x[:, q], v[:, q])
    np.testing.assert_array_equal(xb, xa[:, q])
    np.testing.assert_allclose(vb, va[:, q], rtol=0, atol=1e-14)


# --------------------------------------------------------------------------
# Phantom particles
# --------------------------------------------------------------------------
def _fraction_in_wall(cz, sz, H):
    """Length of the layer [cz - sz, cz + 1 - sz) lying outside [0, H]."""
    lo, hi = cz - sz, cz + 1 - sz
    inside = max(0.0, min(hi, H) - max(lo, 0.0))
    return 1.0 - inside


def test_wall_fraction_geometry(orc):
    """Wall volume fraction of each shifted layer, by interval intersection."""
    H = 9
    p = orc.Params(L=(4, 4, H), walls=True)
    for sz in [-0.5, -0.31, -2.0**-24, 0.0, 2.0**-24, 0.25, 0.5 - 2.0**-24]:
        for cz in range(-1, H + 1):
            exp = _fraction_in_wall(cz, sz, H)
            got = orc.wall_fraction(p, sz, cz)
            if exp >= 1.0 - 1e-15 and got == 0.0:
                continue  # layer entirely inside the wall holds no fluid
            assert abs(got - exp) < 1e-15, (sz, cz, got, exp)


def test_phantom_count_and_velocity_laws(orc):
    """Phantoms: count Poisson(<N_c> f_w), velocities N(0, kT/m) per component."""
    p = orc.Params(density=10.0, kT=2.0, mass=1.0, walls=True, seed=3)
    fw = 0.37
    counts, vel = [], []
    for i in range(4000):
        ph = orc.phantoms(p, i // 500, i % 500, fw)
        counts.append(len(ph))
        vel.append(ph)
    counts = np.array(counts)
    lam = p.density * fw
    ks = np.arange(0, counts.max() + 1)
    obs = np.bincount(counts, minlength=ks.size)
    exp = stats.poisson.pmf(ks, lam) * counts.size
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3
    allv = np.concatenate(vel).ravel()
    assert stats.kstest(allv, stats.norm(0, math.sqrt(p.kT / p.mass)).cdf).pvalue > 1e-3


def test_phantoms_enter_cell_sums(orc):
    """In wall-cut cells the phantoms join the cell: v_cm and the count include
    them (Sec. II, Boundary conditions)."""
    L = (6, 5, 4)
    p = orc.Params(L=L, walls=True, mbs=True, seed=19)
    x, v = synth.box_state(L, seed=23)
    t = 6
    xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, t, x, v)
    s = orc.shift(p, t)
    plane = L[0] * L[1]
    checked = 0
    for c in range(p.ncells):
        idx = np.nonzero(key == c)[0]
        if idx.size == 0:
            continue
        cz = c // plane - 1
        fw = _fraction_in_wall(cz, s[2], L[2])
        ph = orc.phantoms(p, t, c, fw) if fw > 1e-15 else np.zeros((0, 3))
        assert cells[c, 1] == len(ph)
        tot = idx.size + len(ph)
        Vex = [math.fsum(list(vs[k, idx]) + list(ph[:, k])) / tot for k in range(3)]
        np.testing.assert_allclose(cells[c, 2:5], Vex, rtol=0, atol=1e-14)
        checked += len(ph) > 0
    assert checked > 10


# --------------------------------------------------------------------------
# Many steps: Maxwell distribution, conservation, observables
# --------------------------------------------------------------------------
def test_maxwell_from_non_gaussian_start(orc):
    """SRD drives any velocity distribution to Maxwell-Boltzmann at the
    temperature fixed by the (conserved) energy."""
    L = (8, 8, 8)
    p = orc.Params(L=L, seed=37)
    x, v = synth.box_state(L, seed=7, velocity="uniform")
    assert abs(stats.kurtosis(v.ravel(), fisher=False) - 1.8) < 0.05
    x, v = orc.run(p, x, v, 200)
    T = orc.observables(p, v)["T"]
    w = (v - v.mean(axis=1, keepdims=True)).ravel()
    assert stats.kstest(w, stats.norm(0, math.sqrt(T)).cdf).pvalue > 1e-3
    kurt = stats.kurtosis(w, fisher=False)
    assert abs(kurt - 3.0) < 4 * math.sqrt(24.0 / w.size)


def test_energy_and_momentum_conservation_100_steps(orc):
    """Without the thermostat SRD conserves energy and momentum over many steps."""
    L = (8, 8, 8)
    p = orc.Params(L=L, seed=41)
    x, v = synth.box_state(L, seed=17)
    o0 = orc.observables(p, v)
    x, v = orc.run(p, x, v, 100, reorder_every=7)
    o1 = orc.observables(p, v)
    assert abs(o1["E"] - o0["E"]) / o0["E"] < 1e-12
    assert np.abs(o1["P"] - o0["P"]).max() < 1e-10 * math.sqrt(x.shape[1])
    assert o1["N"] == x.shape[1]


def test_observables_against_fsum(orc):
    L = (5, 5, 5)
    p = orc.Params(L=L, mass=1.5)
    _, v = synth.box_state(L, seed=3)
    v = v + 0.3
    o = orc.observables(p, v)
    for k in range(3):
        assert o["P"][k] == pytest.approx(1.5 * math.fsum(v[k]), abs=1e-12)
    assert o["E"] == pytest.approx(0.75 * math.fsum((v ** 2).ravel()), rel=1e-14)
    dv = v - v.mean(axis=1, keepdims=True)
    T = 1.5 * math.fsum((dv ** 2).ravel()) / (3 * (v.shape[1] - 1))
    assert o["T"] == pytest.approx(T, rel=1e-13)


def test_reorder_is_gather(orc):
    rng = np.random.default_rng(1)
    x, v = rng.normal(size=(3, 50)), rng.normal(size=(3, 50))
    perm = rng.permutation(50).astype(np.uint32)
    x2, v2 = orc.reorder(x, v, perm)
    np.testing.assert_array_equal(x2, x[:, perm])
    np.testing.assert_array_equal(v2, v[:, perm])


def test_step_is_composition_of_parts(orc):
    L = (6, 6, 6)
    p = orc.Params(L=L, mbs=True, seed=43)
    x, v = synth.box_state(L, seed=19)
    xs, vs, key, perm, off, v2, _ = _one_step_parts(orc, p, 9, x, v)
    xa, va, ka, pa, oa = orc.step(p, 9, x, v, reorder=True, binning=True)
    np.testing.assert_array_equal(ka, key)
    np.testing.assert_array_equal(pa, perm)
    np.testing.assert_array_equal(oa, off)
    np.testing.assert_array_equal(xa, xs[:, perm])
    np.testing.assert_array_equal(va, v2[:, perm])


# --------------------------------------------------------------------------
# Poiseuille flow: walls + phantoms + gravity + thermostat together
# --------------------------------------------------------------------------
def srd_viscosity(nc, h, alpha, kT=1.0, m=1.0):
    """Kinetic + collisional SRD viscosity with random shift (literature form)."""
    e = nc - 1 + math.exp(-nc)
    kin = nc * kT * h * (5 * nc / (e * (4 - 2 * math.cos(alpha) - 2 * math.cos(2 * alpha))) - 0.5)
    col = m / (18 * h) * e * (1 - math.cos(alpha))
    return kin + col


@pytest.mark.slow
def test_poiseuille_profile(orc):
    """Gravity along x between no-slip walls gives the parabola
    v_x(z) = rho g z (H - z) / (2 eta) (Sec. II, External fields)."""
    L = (8, 8, 16)
    H = L[2]
    g = 0.01
    p = orc.Params(L=L, walls=True, mbs=True, g=(g, 0.0, 0.0), seed=5)
    x, v = synth.box_state(L, seed=13)
    x, v = orc.run(p, x, v, 1500)
    nb = 32
    acc = np.zeros(nb)
    cnt = np.zeros(nb)
    for t in range(1500, 3000):
        x, v = orc.step(p, t, x, v)
        b = np.minimum((x[2] / H * nb).astype(int), nb - 1)
        acc += np.bincount(b, weights=v[0], minlength=nb)
        cnt += np.bincount(b, minlength=nb)
    prof = acc / cnt
    z = (np.arange(nb) + 0.5) * H / nb
    A = np.vstack([z * (H - z), np.ones(nb)]).T
    (a, c), *_ = np.linalg.lstsq(A, prof, rcond=None)
    vmax = a * H * H / 4
    eta_fit = p.density * g / (2 * a)
    eta_th = srd_viscosity(p.density, p.h, p.alpha)
    assert abs(c) < 0.05 * vmax            # no slip at the walls
    assert abs(eta_fit / eta_th - 1) < 0.10
    resid = prof - A @ np.array([a, c])
    assert np.abs(resid).max() < 0.05 * vmax


# --- SRD+a (angular-momentum-conserving variant, Eqs. 3-4) -------------------
def _amc_parts(orc, L, density, t, seed, alpha=np.deg2rad(130.0)):
    """Streamed state, binning and both collisions (plain SRD and SRD+a) of
    one step; positions in the cell frame are frac(x + s) (a = 1)."""
    p = orc.Params(L=L, density=density, seed=seed, alpha=alpha)
    pa = orc.Params(L=L, density=density, seed=seed, alpha=alpha, amc=True)
    x, v = synth.box_state(L, density=density, seed=seed + 100)
    xs, vs, _ = orc.stream(p, x, v)
    key = orc.keys(p, t, xs)
    perm, off = orc.sort(key, p.ncells)
    v_plain = orc.collide(p, t, vs, perm, off)
    v_amc = orc.collide(pa, t, vs, perm, off, x=xs)
    y = xs + orc.shift(p, t)[:, None]
    frame = y - np.floor(y)
    return key, off, frame, vs, v_plain, v_amc


def _cell_L(r, v):
    return np.cross(r.T, v.T).sum(axis=0)


@pytest.mark.parametrize("L,density", [((6, 6, 6), 10.0), ((8, 8, 8), 1.5)])
def test_amc_conserves_angular_momentum(orc, L, density):
    """Eqs. 3-4: SRD+a keeps each cell's momentum and its angular momentum
    about the cell's centre of mass; plain SRD (Eq. 2) does not.  The dilute
    box has many cells of two and three particles."""
    key, off, frame, vs, v_plain, v_amc = _amc_parts(orc, L, density, 3, 12)
    sizes = np.diff(off)
    if density < 2:
        assert (sizes == 2).sum() > 20 and (sizes == 3).sum() > 20
    broken = 0
    for c in np.nonzero(sizes >= 2)[0]:
        idx = np.nonzero(key == c)[0]
        r = frame[:, idx] - frame[:, idx].mean(axis=1, keepdims=True)
        scale = np.abs(vs[:, idx]).sum() * max(1.0, np.abs(r).max())
        L0 = _cell_L(r, vs[:, idx])
        assert np.abs(_cell_L(r, v_amc[:, idx]) - L0).max() <= 1e-12 * scale * idx.size
        dP = np.abs(v_amc[:, idx].sum(axis=1) - vs[:, idx].sum(axis=1)).max()
        assert dP <= 1e-14 * scale * idx.size
        broken += np.abs(_cell_L(r, v_plain[:, idx]) - L0).max() > 1e-3
    assert broken > 0.9 * (sizes >= 2).sum()


def test_amc_correction_is_rigid_rotation(orc):
    """Eqs. 3-4: SRD+a adds to the SRD result a rigid rotation omega x r_ic,
    one omega per cell; a lone particle is left as SRD leaves it.  With the
    conservation pin this fixes omega wherever the inertia tensor is regular."""
    key, off, frame, vs, v_plain, v_amc = _amc_parts(orc, (6, 6, 6), 4.0, 5, 21)
    sizes = np.diff(off)
    for c in np.nonzero(sizes >= 1)[0]:
        idx = np.nonzero(key == c)[0]
        d = v_amc[:, idx] - v_plain[:, idx]
        if idx.size == 1:
            assert np.array_equal(d, np.zeros_like(d))
            continue
        r = frame[:, idx] - frame[:, idx].mean(axis=1, keepdims=True)
        # omega x r = -[r]_x omega: stack the skew matrices and solve by least squares
        A = np.concatenate([np.array([[0.0, rz, -ry], [-rz, 0.0, rx], [ry, -rx, 0.0]])
                            for rx, ry, rz in r.T])
        om, *_ = np.linalg.lstsq(A, d.T.reshape(-1), rcond=None)
        assert np.abs(A @ om - d.T.reshape(-1)).max() <= 1e-12 * max(1.0, np.abs(d).max())


def test_amc_alpha_zero_is_identity(orc):
    """alpha = 0: D = 1, so the torque and omega vanish and SRD+a equals SRD."""
    key, off, frame, vs, v_plain, v_amc = _amc_parts(orc, (4, 4, 4), 10.0, 2, 31, alpha=0.0)
    assert np.array_equal(v_amc, v_plain)
    np.testing.assert_allclose(v_amc, vs, rtol=0, atol=1e-14)


def test_amc_refused_with_walls(orc):
    """SRD+a is taken to be defined for periodic boxes and slip walls (phantom
    particles carry no positions); the oracle refuses no-slip walls and a
    missing x."""
    x, v = synth.box_state((4, 4, 4), seed=3)
    perm, off = orc.sort(orc.keys(orc.Params(L=(4, 4, 4)), 0, x), 64)
    with pytest.raises(ValueError):
        orc.collide(orc.Params(L=(4, 4, 4), amc=True), 0, v, perm, off)
    with pytest.raises(ValueError):
        orc.step(orc.Params(L=(4, 4, 4), amc=True, walls=True), 0, x, v)
    orc.step(orc.Params(L=(4, 4, 4), amc=True, walls=True, slip=True), 0, x, v)


def test_amc_with_slip_walls_conserves_angular_momentum(orc):
    """Eqs. 3-4 next to slip walls (cut cells hold fluid particles only): per
    cell, momentum and angular momentum about the centre of mass are kept."""
    L = (6, 6, 5)
    t = 3
    pa = orc.Params(L=L, walls=True, slip=True, amc=True, seed=19)
    x, v = synth.box_state(L, seed=23)
    v *= 2.0
    xs, vs, nb = orc.stream(pa, x, v)
    assert nb > 20
    key = orc.keys(pa, t, xs)
    perm, off = orc.sort(key, pa.ncells)
    va = orc.collide(pa, t, vs, perm, off, x=xs)
    y = xs + orc.shift(pa, t)[:, None]
    fr = y - np.floor(y)
    checked = 0
    for c in np.nonzero(np.diff(off) >= 2)[0]:
        idx = perm[off[c]:off[c + 1]]
        r = fr[:, idx] - fr[:, idx].mean(axis=1, keepdims=True)
        scale = np.abs(vs[:, idx]).sum()
        assert np.abs(_cell_L(r, va[:, idx]) - _cell_L(r, vs[:, idx])).max() <= 1e-12 * scale
        assert np.abs(va[:, idx].sum(axis=1) - vs[:, idx].sum(axis=1)).max() <= 1e-13 * scale
        checked += 1
    assert checked > 100


def test_amc_with_thermostat(orc):
    """SRD+a with MBS: per cell, the corrected relative velocities of SRD+a
    scaled by one factor kappa whose result has relative kinetic energy equal
    to the drawn E_k (Gamma(3(N_c-1)/2, kT) law); momentum is conserved and
    the angular momentum about the centre of mass is scaled by kappa."""
    L = (10, 10, 10)
    t = 4
    pa = orc.Params(L=L, amc=True, seed=17, kT=1.3)
    pm = orc.Params(L=L, amc=True, mbs=True, seed=17, kT=1.3)
    x, v = synth.box_state(L, seed=91, kT=0.7)
    xs, vs, _ = orc.stream(pa, x, v)
    key = orc.keys(pa, t, xs)
    perm, off = orc.sort(key, pa.ncells)
    va = orc.collide(pa, t, vs, perm, off, x=xs)
    vm, cells = orc.collide(pm, t, vs, perm, off, cells=True, x=xs)
    y = xs + orc.shift(pa, t)[:, None]
    fr = y - np.floor(y)
    sel = np.nonzero(cells[:, 0] >= 2)[0]
    for c in sel:
        idx = perm[off[c]:off[c + 1]]
        V = cells[c, 2:5][:, None]
        scale = np.abs(vs[:, idx]).sum()
        assert np.abs(vm[:, idx].sum(axis=1) - vs[:, idx].sum(axis=1)).max() <= 1e-14 * scale
        da, dm = va[:, idx] - V, vm[:, idx] - V
        kappa = math.sqrt(2 * cells[c, 10] / (da ** 2).sum())
        np.testing.assert_allclose(dm, kappa * da, rtol=0, atol=1e-13 * np.abs(dm).max())
        assert abs((dm ** 2).sum() - 2 * cells[c, 10]) <= 1e-12 * cells[c, 10]
        r = fr[:, idx] - fr[:, idx].mean(axis=1, keepdims=True)
        L0 = _cell_L(r, vs[:, idx])
        np.testing.assert_allclose(_cell_L(r, vm[:, idx]), kappa * L0, rtol=0,
                                   atol=1e-12 * scale)
    np.testing.assert_allclose(cells[sel, 15], 2 * cells[sel, 10], rtol=1e-12)
    u = stats.gamma.cdf(cells[sel, 10] / pm.kT, 1.5 * (cells[sel, 0] - 1))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


# --- fixed-point cell sums (Sec. III.C) ---------------------------------------
def _fixed_state(L, seed):
    """Maxwellian velocities with a few tiny ones, so that some terms are not
    multiples of 2^-80 and the truncation rule matters."""
    x, v = synth.box_state(L, seed=seed)
    rng = np.random.default_rng(seed + 1)
    tiny = rng.random(x.shape[1]) < 0.05
    v[:, tiny] = rng.normal(size=(3, tiny.sum())) * 1e-13
    return x, v


def _exact_fixed_sum(terms):
    """The definition with Python integers: sum of trunc(t 2^80), rounded once
    (int / int is correctly rounded) and scaled by 2^-80."""
    return sum(int(t * 2 ** 80) for t in terms) / 2 ** 80


@pytest.mark.parametrize("vscale", [1.0, 1e-13])
def test_fixed_sums_exact(orc, vscale):
    """Sec. III.C: with fixed-point sums, each cell's momentum, mean velocity
    and kinetic energy equal the exact integer definition bit for bit.  With
    tiny velocities the sums are far below 1, so that the truncation of each
    term to the 2^-80 grid shows in the rounded result."""
    L = (6, 6, 6)
    p = orc.Params(L=L, mbs=True, fixed=True, mass=1.3, seed=41)
    x, v = _fixed_state(L, 43)
    v *= vscale
    xs, vs, key, perm, off, v2, cells = _one_step_parts(orc, p, 3, x, v)
    checked = 0
    for c in range(p.ncells):
        idx = perm[off[c]:off[c + 1]]
        if idx.size == 0:
            continue
        m = p.mass
        P = [_exact_fixed_sum(float(m * vv) for vv in vs[k, idx]) for k in range(3)]
        assert [cells[c, 12 + k] for k in range(3)] == P
        V = [Pk / (idx.size * m) for Pk in P]
        assert [cells[c, 2 + k] for k in range(3)] == V
        terms = []
        for i in idx:
            dx, dy, dz = (float(vs[k, i]) - V[k] for k in range(3))
            terms.append(m * (dx * dx + dy * dy + dz * dz))
        assert cells[c, 5] == _exact_fixed_sum(terms)
        checked += 1
    assert checked > 0.9 * p.ncells


@pytest.mark.parametrize("amc", [False, True])
def test_fixed_sums_order_independent(orc, amc):
    """Sec. III.C: with fixed-point sums the trajectory does not depend on the
    order in which particles are stored; with FP64 sums it does (at rounding
    level)."""
    L = (5, 6, 7)
    x, v = _fixed_state(L, 47)
    perm = np.random.default_rng(5).permutation(x.shape[1])
    inv = np.argsort(perm)
    runs = {}
    for fixed in (False, True):
        p = orc.Params(L=L, mbs=True, amc=amc, fixed=fixed, seed=53)
        xa, va = orc.run(p, x, v, 3)
        xb, vb = orc.run(p, x[:, perm], v[:, perm], 3)
        runs[fixed] = (np.array_equal(xa, xb[:, inv]), np.array_equal(va, vb[:, inv]))
    assert runs[True] == (True, True)
    assert runs[False][1] is False


def test_fixed_sums_range(orc):
    """A summand outside |x| < 2^37 is refused in fixed-point mode."""
    L = (4, 4, 4)
    x, v = synth.box_state(L, seed=3)
    v[0, 7] = 2.0 ** 19  # its kinetic-energy term is about 2^38
    refused = False
    try:
        orc.step(orc.Params(L=L, fixed=True), 0, x, v)
    except ValueError:
        refused = True
    assert refused
    orc.step(orc.Params(L=L), 0, x, v)


# --- slip walls and moving no-slip walls (Sec. II, Boundary conditions) -------
def test_moving_wall_bounce_is_galilean(orc):
    """A no-slip wall moving with velocity u along x bounces particles as a wall
    at rest does in the wall's own frame (Galilean invariance): streaming with
    the moving wall equals streaming v - u past a resting wall, shifted back by
    u h and u.  The wall at z = H moves with +U, the wall at z = 0 with -U."""
    L = (8, 8, 6)
    U = 0.7
    x, v = synth.box_state(L, n=5000, seed=19)
    v *= 3.0
    pm = orc.Params(L=L, h=0.5, walls=True, uwall=U)
    ps = orc.Params(L=L, h=0.5, walls=True)
    x2, v2, nb = orc.stream(pm, x, v)
    zend = x[2] + pm.h * v[2]
    for sel, u in ((zend < 0, -U), (zend > L[2], U)):
        assert sel.sum() > 50
        shift = np.array([u, 0.0, 0.0])[:, None]
        xr, vr, _ = orc.stream(ps, x[:, sel], v[:, sel] - shift)
        np.testing.assert_allclose(v2[:, sel], vr + shift, rtol=0, atol=1e-14)
        xe = xr + pm.h * shift
        d = np.abs(x2[:, sel] - xe)
        d[0] = d[0] % L[0]
        d[0] = np.minimum(d[0], L[0] - d[0])
        assert d.max() < 1e-12
    rest = (zend >= 0) & (zend <= L[2])
    xs, vs, _ = orc.stream(ps, x[:, rest], v[:, rest])
    np.testing.assert_array_equal(x2[:, rest], xs)
    np.testing.assert_array_equal(v2[:, rest], vs)


def test_slip_walls_reflect_specularly(orc):
    """Slip walls: a crossing particle is mirrored in z (z -> -z_end or
    2H - z_end) with v_z reversed; x, y and v_x, v_y are those of free
    flight."""
    L = (8, 8, 6)
    p = orc.Params(L=L, h=0.5, walls=True, slip=True)
    x, v = synth.box_state(L, n=5000, seed=29)
    v *= 3.0
    x2, v2, nb = orc.stream(p, x, v)
    zend = x[2] + p.h * v[2]
    bot, top = zend < 0, zend > L[2]
    assert nb == int((bot | top).sum()) > 100
    np.testing.assert_allclose(x2[2, bot], -zend[bot], rtol=0, atol=1e-13)
    np.testing.assert_allclose(x2[2, top], 2 * L[2] - zend[top], rtol=0, atol=1e-13)
    np.testing.assert_array_equal(v2[:2], v[:2])
    np.testing.assert_array_equal(v2[2, bot | top], -v[2, bot | top])
    free = orc.Params(L=(8, 8, 6), h=0.5)
    xf, _, _ = orc.stream(free, x, v)
    np.testing.assert_array_equal(x2[:2], xf[:2])


def test_slip_walls_exert_no_tangential_force(orc):
    """With slip walls (no phantoms) a body force g along x raises the total
    momentum by N m g h per step exactly (to rounding); no-slip walls exchange
    momentum with the fluid."""
    L = (6, 6, 8)
    x, v = synth.box_state(L, seed=37)
    n = x.shape[1]
    g = 0.01
    out = {}
    for slip in (True, False):
        p = orc.Params(L=L, walls=True, slip=slip, mbs=True, g=(g, 0.0, 0.0), seed=3)
        x1, v1 = orc.run(p, x, v, 30)
        out[slip] = v1[0].sum() - v[0].sum()
    expect = n * g * 0.1 * 30
    assert abs(out[True] - expect) < 1e-9 * n
    assert abs(out[False] - expect) > 1.0


def test_couette_profile(orc):
    """No-slip walls moving with +-U along x: the time-averaged steady profile
    v_x(z) is linear through zero at mid-height with slope close to 2U/H (the
    phantoms keep the slip at the walls small)."""
    L = (6, 6, 10)
    U = 0.5
    p = orc.Params(L=L, walls=True, mbs=True, uwall=U, seed=11)
    x, v = synth.box_state(L, seed=45)
    x, v = orc.run(p, x, v, 500)
    nb = 20
    acc = np.zeros(nb)
    cnt = np.zeros(nb)
    for t in range(500, 1700, 4):
        x, v = orc.run(p, x, v, 4, t0=t)
        b = np.minimum((x[2] / L[2] * nb).astype(int), nb - 1)
        acc += np.bincount(b, v[0], nb)
        cnt += np.bincount(b, minlength=nb)
    z = (np.arange(nb) + 0.5) * L[2] / nb
    prof = acc / cnt
    slope, icpt = np.polyfit(z - L[2] / 2, prof, 1)
    resid = prof - (slope * (z - L[2] / 2) + icpt)
    r2 = 1 - (resid ** 2).sum() / ((prof - prof.mean()) ** 2).sum()
    print(f"Couette: slope {slope:.4f} (2U/H = {2 * U / L[2]:.4f}), intercept {icpt:.4f}, R2 {r2:.4f}")
    assert abs(slope / (2 * U / L[2]) - 1) < 0.1
    assert abs(icpt) < 0.02 and r2 > 0.98


# --- Lees-Edwards shear of a periodic box (Sec. II, boundary conditions) ------
def _le_offset(U, t_end, h, Lx):
    return (U * t_end * h) % Lx


def test_lees_edwards_stream(orc):
    """A particle through the upper z face re-enters at the bottom displaced by
    -d along x with v_x - U (it is the image of one below the box); through
    the lower face +d and + U; d = (U (t+1) h) mod L_x."""
    L = (8, 6, 6)
    U, t = 0.9, 13
    p = orc.Params(L=L, h=0.5, le_u=U)
    x, v = synth.box_state(L, n=4000, seed=53)
    v *= 3.0
    x2, v2, _ = orc.stream(p, x, v, t=t)
    free, _, _ = orc.stream(orc.Params(L=L, h=0.5), x, v, t=t)
    zend = x[2] + p.h * v[2]
    up, down = zend >= L[2], zend < 0
    assert up.sum() > 100 and down.sum() > 100
    d = _le_offset(U, t + 1, p.h, L[0])
    for sel, sgn in ((up, -1.0), (down, 1.0)):
        ex = (x[0, sel] + p.h * v[0, sel] + sgn * d) % L[0]
        dd = np.abs(x2[0, sel] - ex)
        assert np.minimum(dd, L[0] - dd).max() < 1e-12
        np.testing.assert_allclose(v2[0, sel], v[0, sel] + sgn * U, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(x2[1:], free[1:])
    rest = ~(up | down)
    np.testing.assert_array_equal(x2[:, rest], free[:, rest])
    np.testing.assert_array_equal(v2[:, rest], v[:, rest])


def test_lees_edwards_keys_use_the_image(orc):
    """A particle whose shifted cell lies across a z face is binned as its image
    on the other side: the plain periodic keys of (x -/+ d, y, z -/+ L_z)."""
    L = (8, 6, 6)
    U, t = 0.7, 21
    p = orc.Params(L=L, le_u=U, seed=9)
    plain = orc.Params(L=L, seed=9)
    x, _ = synth.box_state(L, n=20000, seed=59)
    s = orc.shift(p, t)
    d = _le_offset(U, t + 1, p.h, L[0])
    cz = np.floor(x[2] + s[2])
    xm = x.copy()
    top, bot = cz >= L[2], cz < 0
    assert top.sum() + bot.sum() > 100
    xm[0, top] = (x[0, top] - d) % L[0]
    xm[2, top] = x[2, top] - L[2]
    xm[0, bot] = (x[0, bot] + d) % L[0]
    xm[2, bot] = x[2, bot] + L[2]
    np.testing.assert_array_equal(orc.keys(p, t, x), orc.keys(plain, t, xm))


def test_lees_edwards_momentum_budget(orc):
    """Collisions conserve momentum in each cell's frame, so a step changes the
    total x momentum only through the face crossings: by U (n_down - n_up)."""
    L = (8, 6, 6)
    U, t = 0.6, 4
    p = orc.Params(L=L, le_u=U, mbs=True, seed=15)
    x, v = synth.box_state(L, seed=61)
    v *= 2.0
    zend = x[2] + p.h * v[2]
    n_up, n_down = int((zend >= L[2]).sum()), int((zend < 0).sum())
    assert n_up + n_down > 20
    x2, v2 = orc.step(p, t, x, v)
    dP = v2[0].sum() - v[0].sum()
    assert abs(dP - U * (n_down - n_up)) < 1e-11 * x.shape[1]


def test_lees_edwards_shear_profile(orc):
    """Steady Lees-Edwards shear: the averaged v_x(z) is linear with slope
    U / L_z through the whole box (no walls, so no slip)."""
    L = (6, 6, 12)
    U = 0.6
    p = orc.Params(L=L, le_u=U, mbs=True, seed=21)
    x, v = synth.box_state(L, seed=63)
    x, v = orc.run(p, x, v, 400)
    nb = 12
    acc = np.zeros(nb)
    cnt = np.zeros(nb)
    for t in range(400, 1600, 4):
        x, v = orc.run(p, x, v, 4, t0=t)
        b = np.minimum((x[2] / L[2] * nb).astype(int), nb - 1)
        acc += np.bincount(b, v[0], nb)
        cnt += np.bincount(b, minlength=nb)
    z = (np.arange(nb) + 0.5) * L[2] / nb
    slope, icpt = np.polyfit(z, acc / cnt, 1)
    print(f"Lees-Edwards: slope {slope:.4f} (U/L_z = {U / L[2]:.4f})")
    assert abs(slope / (U / L[2]) - 1) < 0.05


def test_amc_lees_edwards_conserves_angular_momentum(orc):
    """SRD+a under Lees-Edwards shear: a cell across a z face holds particles
    seen as their images (x -/+ d, v_x -/+ U); in that frame each cell keeps
    its momentum and its angular momentum about the centre of mass."""
    L = (6, 6, 6)
    U, t = 0.7, 5
    p = orc.Params(L=L, le_u=U, amc=True, seed=31)
    x, v = synth.box_state(L, seed=67)
    xs, vs, _ = orc.stream(p, x, v, t=t)
    key = orc.keys(p, t, xs)
    perm, off = orc.sort(key, p.ncells)
    va = orc.collide(p, t, vs, perm, off, x=xs)
    s = orc.shift(p, t)
    d = _le_offset(U, t + 1, p.h, L[0])
    cz = np.floor(xs[2] + s[2])
    side = np.where(cz < 0, 1.0, np.where(cz >= L[2], -1.0, 0.0))
    xm = xs.copy()
    xm[0] += side * d
    y = xm + s[:, None]
    fr = y - np.floor(y)
    vf0, vf1 = vs.copy(), va.copy()
    vf0[0] += side * U
    vf1[0] += side * U
    crossing = 0
    for c in np.nonzero(np.diff(off) >= 2)[0]:
        idx = perm[off[c]:off[c + 1]]
        crossing += bool(np.any(side[idx] != 0))
        r = fr[:, idx] - fr[:, idx].mean(axis=1, keepdims=True)
        scale = np.abs(vf0[:, idx]).sum()
        assert np.abs(_cell_L(r, vf1[:, idx]) - _cell_L(r, vf0[:, idx])).max() <= 1e-12 * scale
        assert np.abs(vf1[:, idx].sum(axis=1) - vf0[:, idx].sum(axis=1)).max() <= 1e-13 * scale
    assert crossing > 10
