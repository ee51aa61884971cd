"""Parity at size for the reduced-precision forms and the batched form.

FP32 and split (positions as an integer cell plus an FP32 offset, FP32
velocities; reduced precision for particle data, Sec. III.G), one step from a
stored state:
  * binning bit-identical given the GPU's post-stream positions (keys of
    every particle, the stable permutation and the offsets);
  * streaming against the FP64 oracle run from the same stored state, within
    the rounding bound of the form (stated per test);
  * the collision, fed the GPU's post-stream state, within e <= 2e-6 of the
    FP64 oracle, e = |v_gpu - v_orc| / max(|v_orc|, sqrt(kT/m)).
FP64: positions, keys, permutation and offsets bit-identical; e <= 1e-12.

Boxes: the packing limits of the split form's cell index (2048 cells along x
or y, 1024 along z), the 256^3 box with the thermostat (FP32 and split), the
512^3 box of the precision comparison (FP64 and split; velocities on sampled
cells, binning structure over all 1.34e9 particles), and the batched
ensemble of 64 uneven boxes (FP64 and split).  The large boxes run in the
tiling chosen by the library's autotuner, as the benchmark does.
"""
import math
import time

import numpy as np
import pytest

import oracle as orc
import synth

pytestmark = pytest.mark.gpu

DEG = math.pi / 180.0
# split form: an offset in [0, 1) advanced by fmaf(h_f32, v, o) lies below 2,
# so one rounding is at most half an ulp of [1, 2) = 2^-24 cells; the step
# h rounded to FP32 adds |h_f32 - h| |v| < 1.5e-9 |v| (speeds here < 10)
SPLIT_STREAM_BAR = 2.0 ** -24 + 2e-8


def fp32_stream_bar(L):
    """FP32 absolute positions: x + h v is rounded once in FP32 before the
    periodic wrap; the value lies below L + 1, so the error is at most half
    an ulp of L + 1 (plus the FP32 rounding of h, < 1.5e-9 |v|)."""
    return 0.5 * float(np.spacing(np.float32(max(L) + 1))) + 2e-8


@pytest.fixture(scope="module")
def mpc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_15236_amd as m
    m.lib()
    return m


def oparams(box):
    return orc.Params(L=box["L"], h=box["h"], alpha=box["alpha"], kT=box["kT"],
                      mass=box["mass"], density=box["density"], seed=box["seed"],
                      mbs=box.get("mbs", False), walls=box.get("walls", False),
                      g=box.get("g", (0.0, 0.0, 0.0)))


def rel_err(vg, vo, box):
    floor = math.sqrt(box["kT"] / box["mass"])
    return np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), floor)


def report(name, e):
    print(f"{name}: max e = {e.max():.3e}, p99 = {np.quantile(e, 0.99):.3e}, n = {e.size}",
          flush=True)


def periodic_dist(a, b, L, walls=False):
    d = np.abs(a - b)
    for k in range(3):
        if not (walls and k == 2):
            d[k] = np.minimum(d[k], L[k] - d[k])
    return d


def check_binning_structure(kg, pg, og, ncell):
    """The stable counting sort is fixed by the keys: offsets are the
    exclusive prefix of the per-cell counts, the permutation lists every
    particle once, in non-decreasing key and ascending index inside a cell.
    Holds at any size; used where the oracle cannot sort the whole box."""
    n = kg.size
    assert og[0] == 0 and int(og[-1]) == n
    assert np.all(og[1:] >= og[:-1])
    cnt = np.bincount(kg, minlength=ncell)
    assert cnt.size == ncell
    assert np.array_equal(cnt, (og[1:].astype(np.int64) - og[:-1]))
    del cnt
    seen = np.zeros(n, dtype=bool)
    seen[pg] = True
    assert seen.all()
    del seen
    kp = kg[pg]
    assert np.all(kp[1:] >= kp[:-1])
    same = kp[1:] == kp[:-1]
    del kp
    assert np.all(pg[1:][same] > pg[:-1][same])


def sampled_cells(og, ncell, count, seed):
    rng = np.random.default_rng(seed)
    cells = np.sort(rng.choice(ncell, size=count, replace=False))
    counts = (og[cells + 1].astype(np.int64) - og[cells])
    return cells, counts


def sample_offsets(ncell, cells, counts):
    off = np.zeros(ncell + 1, dtype=np.uint32)
    cnt = np.zeros(ncell, dtype=np.int64)
    cnt[cells] = counts
    off[1:] = np.cumsum(cnt).astype(np.uint32)
    return off


def one_step_reduced(mpc, box, form, R, t0, x, v, tune=False):
    """Set (x, v), run step t0 on the GPU; return the stored pre-step state,
    the post-step state (caller's order) and the binning."""
    with mpc.Sim(box, form=form, reorder_every=R) as sim:
        sim.set_state(x, v)
        if tune:
            sim.step(1)
            sim.autotune(2)   # restores the state and the step counter
            sim.set_state(x, v)
        x0, v0 = sim.get_state()
        sim.set_step(t0)
        sim.step(1)
        x1, v1 = sim.get_state()
        kg, pg, og = sim.get_binning()
        tiling = sim.get_tiling()
    return x0, v0, x1, v1, kg, pg, og, tiling


def check_reduced_full(box, form, R, t0, x0, v0, x1, v1, kg, pg, og, sample_cells=None):
    """All particles: stream bound, binning; velocities on all cells or on a
    sample of cells."""
    p = oparams(box)
    L = box["L"]
    walls = box.get("walls", False)
    sorted_out = R > 0 and (t0 + 1) % R == 0
    xs, vs, _ = orc.stream(p, x0, v0)
    if sorted_out:  # back to the pre-step order, particle by particle
        x1u = np.empty_like(x1)
        v1u = np.empty_like(v1)
        x1u[:, pg] = x1
        v1u[:, pg] = v1
    else:
        x1u, v1u = x1, v1
    dx = periodic_dist(x1u, xs, L, walls)
    bar = SPLIT_STREAM_BAR if form == "split" else fp32_stream_bar(L)
    bounced = (np.any(np.sign(vs) != np.sign(v0), axis=0) if walls
               else np.zeros(x0.shape[1], dtype=bool))
    free = ~bounced
    print(f"{form} {L}: max stream error {dx[:, free].max():.3e} cells (bar {bar:.3e}), "
          f"{bounced.sum()} bounced", flush=True)
    assert dx[:, free].max() <= bar
    if bounced.any():
        # FP32 absolute positions: the crossing time (z - H) / v_z inherits
        # ulp(H) / |v_z|; the split form bounces in FP64 from the exact
        # position and rounds the new offset once
        assert dx[:, bounced].max() <= (1e-4 if form == "fp32" else bar)
    del dx, xs
    ko = orc.keys(p, t0, x1u)
    np.testing.assert_array_equal(kg, ko)
    po, oo = orc.sort(ko, p.ncells)
    del ko
    np.testing.assert_array_equal(og, oo)
    np.testing.assert_array_equal(pg, po)
    vpre = v0
    if walls:
        vpre = v0.copy()
        flipped = np.all(np.sign(vs) != np.sign(v0), axis=0) & np.any(v0 != 0, axis=0)
        vpre[:, flipped] = -v0[:, flipped]
    if sample_cells is None:
        vo = orc.collide(p, t0, vpre, po, oo)
        e = rel_err(v1u, vo, box)
    else:
        cells, counts = sampled_cells(oo, p.ncells, sample_cells, seed=7)
        members = np.concatenate([po[oo[c]:oo[c + 1]] for c in cells]).astype(np.int64)
        off_s = sample_offsets(p.ncells, cells, counts)
        vo = orc.collide(p, t0, np.ascontiguousarray(vpre[:, members]),
                         np.arange(members.size, dtype=np.uint32), off_s)
        e = rel_err(v1u[:, members], vo, box)
    report(f"{form} {L} collision", e)
    assert e.max() <= 2e-6


def c2_like(L, **kw):
    b = dict(L=tuple(L), h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=10.0, seed=1,
             mbs=True, walls=False, g=(0.0, 0.0, 0.0))
    b.update(kw)
    return b


@pytest.mark.parametrize("L,walls", [((2048, 8, 8), False), ((8, 2048, 8), False),
                                     ((8, 8, 1024), False), ((8, 8, 1023), True)])
def test_split_packing_limits(mpc, L, walls):
    """The split form's packed cell index (11 bits x, 11 bits y, 10 bits z)
    at the largest extents it accepts."""
    box = c2_like(L, walls=walls, g=(1e-3, 0.0, 0.0) if walls else (0.0, 0.0, 0.0), seed=3)
    print(f"case split L={L} walls={walls}", flush=True)
    x, v = synth.box_state(L, seed=41)
    t0 = 6
    x0, v0, x1, v1, kg, pg, og, _ = one_step_reduced(mpc, box, "split", 1, t0, x, v)
    # the largest cell coordinate along the long axis is occupied
    k = int(np.argmax(L))
    assert np.floor(x1[k]).max() >= L[k] - 1
    check_reduced_full(box, "split", 1, t0, x0, v0, x1, v1, kg, pg, og)


@pytest.mark.parametrize("form", ["fp32", "split"])
def test_reduced_full_size_256(mpc, form):
    """The 256^3 box with the thermostat, 10 per cell (167,772,160
    particles), reorder step of R = 20, autotuned tiling: stream bound and
    binning for every particle, velocities on 2000 sampled cells."""
    box = synth.config("C2")
    t_start = time.time()
    x, v = synth.box_state(box["L"], seed=2025)
    print(f"case {form} 256^3: state made in {time.time() - t_start:.1f} s", flush=True)
    x0, v0, x1, v1, kg, pg, og, tiling = one_step_reduced(mpc, box, form, 20, 19, x, v,
                                                          tune=True)
    del x, v
    print(f"GPU step done at {time.time() - t_start:.1f} s, tiling {tiling}", flush=True)
    check_reduced_full(box, form, 20, 19, x0, v0, x1, v1, kg, pg, og, sample_cells=2000)
    print(f"checked at {time.time() - t_start:.1f} s", flush=True)


@pytest.mark.parametrize("form", ["fp64", "split"])
def test_c3_512_sampled(mpc, form):
    """The 512^3 box of the precision comparison (1,342,177,280 particles,
    plain SRD), device-initialised state, autotuned tiling, one step.  The
    binning's structure is checked over all particles; for the particles of
    3000 sampled cells: the stored pre-step state (re-created by the
    deterministic device initialiser), streaming against the FP64 oracle,
    their keys against the oracle's keys of the GPU's post-stream positions,
    and their velocities against the oracle's collision of those cells."""
    box = synth.config("C3")
    L = box["L"]
    t0 = 7
    t_start = time.time()
    print(f"case C3 {form}", flush=True)
    p = oparams(box)
    with mpc.Sim(box, form=form, reorder_every=0) as sim:
        n = sim.n()
        sim.init_state(3)
        sim.step(1)
        sim.autotune(2)
        sim.init_state(3)
        sim.set_step(t0)
        sim.step(1)
        kg, pg, og = sim.get_binning()
        print(f"GPU step at {time.time() - t_start:.1f} s, tiling {sim.get_tiling()}", flush=True)
        cells, counts = sampled_cells(og, p.ncells, 3000, seed=11)
        members = np.concatenate([pg[og[c]:og[c + 1]] for c in cells]).astype(np.int64)
        x1, v1 = sim.get_particles(members)      # R = 0: logical indices are kept
        sim.init_state(3)
        sim.set_step(t0)
        x0, v0 = sim.get_particles(members)
    print(f"{members.size} sampled particles at {time.time() - t_start:.1f} s", flush=True)
    check_binning_structure(kg, pg, og, p.ncells)
    print(f"binning structure of {n} particles at {time.time() - t_start:.1f} s", flush=True)
    xs, vs, _ = orc.stream(p, x0, v0)
    if form == "fp64":
        np.testing.assert_array_equal(x1, xs)
    else:
        dx = periodic_dist(x1, xs, L)
        print(f"split: max stream error {dx.max():.3e} cells", flush=True)
        assert dx.max() <= SPLIT_STREAM_BAR
    ko = orc.keys(p, t0, x1)
    np.testing.assert_array_equal(kg[members], ko)
    np.testing.assert_array_equal(ko, np.repeat(cells, counts).astype(np.uint32))
    off_s = sample_offsets(p.ncells, cells, counts)
    vo = orc.collide(p, t0, vs, np.arange(members.size, dtype=np.uint32), off_s)
    e = rel_err(v1, vo, box)
    report(f"C3 {form} collision", e)
    assert e.max() <= (1e-12 if form == "fp64" else 2e-6)


def check_fp64_box(b, t0, R, x, v, xg, vg, bins):
    sorted_out = R > 0 and (t0 + 1) % R == 0
    xo, vo, ko, po, oo = orc.step(oparams(b), t0, x, v, reorder=sorted_out, binning=True)
    np.testing.assert_array_equal(bins[0], ko)
    np.testing.assert_array_equal(bins[1], po)
    np.testing.assert_array_equal(bins[2], oo)
    np.testing.assert_array_equal(xg, xo)
    return rel_err(vg, vo, b)


@pytest.mark.parametrize("form,nbox,lmin,lmax", [("split", 6, 6, 15), ("fp64", 64, 16, 96),
                                                 ("split", 64, 16, 96)])
def test_batched(mpc, form, nbox, lmin, lmax):
    """Boxes of uneven sizes, densities, angles and temperatures advanced
    together equal each box stepped alone by the oracle (64 boxes with edges
    16..96: the batched ensemble's scale, about 1.3e8 particles)."""
    boxes = synth.batch_boxes(nbox, seed=4, lmin=lmin, lmax=lmax)
    t_start = time.time()
    print(f"case batched {form} nbox={nbox}", flush=True)
    states = [synth.box_state(b["L"], density=b["density"], kT=b["kT"], seed=100 + i)
              for i, b in enumerate(boxes)]
    t0 = 3
    R = 1
    with mpc.Sim(boxes, form=form, reorder_every=R) as sim:
        for i, (x, v) in enumerate(states):
            sim.set_state(x, v, box=i)
        if nbox > 8:
            sim.step(1)
            sim.autotune(2)
            for i, (x, v) in enumerate(states):
                sim.set_state(x, v, box=i)
        pre = [sim.get_state(box=i) for i in range(nbox)] if form != "fp64" else None
        sim.set_step(t0)
        sim.step(1)
        outs = [sim.get_state(box=i) for i in range(nbox)]
        bins = [sim.get_binning(box=i) for i in range(nbox)]
    ntot = sum(s[0].shape[1] for s in states)
    print(f"{ntot} particles stepped at {time.time() - t_start:.1f} s", flush=True)
    worst = 0.0
    for i, b in enumerate(boxes):
        if form == "fp64":
            e = check_fp64_box(b, t0, R, states[i][0], states[i][1], outs[i][0], outs[i][1],
                               bins[i])
            assert e.max() <= 1e-12, (i, e.max())
            worst = max(worst, float(e.max()))
        else:
            check_reduced_full(b, form, R, t0, pre[i][0], pre[i][1], outs[i][0], outs[i][1],
                               *bins[i])
    print(f"batched {form}: {nbox} boxes checked at {time.time() - t_start:.1f} s"
          + (f", max e = {worst:.3e}" if form == "fp64" else ""), flush=True)
