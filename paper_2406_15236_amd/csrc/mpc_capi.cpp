// mpc_capi.cpp -- host side of the C ABI declared in include/mpc.h: parameter
// validation, workspace planning, tile tables, step sequencing (direct
// launches or a replayed hipGraph of one step), state transfer, observables.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "mpc.h"
#include "mpc_internal.h"

using namespace mpc;

namespace {

constexpr uint64_t kMaxIndex = 0x7fffffffull;  // particle and cell indices stay below 2^31
constexpr int64_t kStateChunk = int64_t(1) << 22;  // particles per host staging chunk
constexpr int kMinTileCells = 4;
constexpr int32_t kMaxGraphSteps = 1000;  // steps captured in one graph
static_assert(MPC_MAX_CELL_PARTICLES == kTileCap, "the ABI's cell limit is one collide pass");

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BoxPlan {
  uint64_t n, ncell;
  int nlz;
};

struct Plan {
  std::vector<BoxPlan> box;
  uint64_t ntot = 0, ctot = 0, cpad = 0;
  uint32_t nscan = 0;
  uint64_t max_tiles = 0, npblocks = 0;
  size_t rec = 0;  // bytes per particle record
  bool split = false;
  // byte offsets in the workspace: records of the two state buffers and, for
  // FP64 and FP32, their logical-index arrays (the split record holds its id)
  size_t off_rec[2] = {}, off_id[2] = {};
  size_t off_rank = 0, off_phs = 0;
  size_t off_key = 0, off_perm = 0, off_hist = 0, off_offset = 0, off_scan = 0, off_ctrl = 0,
         off_boxes = 0, off_tiles = 0, off_pblocks = 0, off_partials = 0, off_vmean = 0,
         off_draws = 0;
  size_t total = 0;
};

int validate(const mpc_params* p, int32_t nbox, std::string* why) {
  if (!p || nbox < 1 || nbox > MPC_MAX_BOXES) {
    *why = "need 1..MPC_MAX_BOXES boxes";
    return MPC_EINVAL;
  }
  for (int32_t b = 0; b < nbox; ++b) {
    const mpc_params& q = p[b];
    char msg[160];
    auto bad = [&](const char* what) {
      snprintf(msg, sizeof msg, "box %d: %s", b, what);
      *why = msg;
      return MPC_EINVAL;
    };
    if (q.form < MPC_FP64 || q.form > MPC_SPLIT32) return bad("unknown form");
    if (q.flags & ~(uint32_t)(MPC_MBS | MPC_WALLS_Z | MPC_SLIP | MPC_AMC | MPC_FIXED_SUMS))
      return bad("unknown flags");
    if ((q.flags & MPC_SLIP) && !(q.flags & MPC_WALLS_Z)) return bad("MPC_SLIP needs MPC_WALLS_Z");
    if (!isfinite(q.wall_u)) return bad("wall_u must be finite");
    if (q.wall_u != 0.0 && (!(q.flags & MPC_WALLS_Z) || (q.flags & MPC_SLIP)))
      return bad("wall_u needs no-slip walls (MPC_WALLS_Z without MPC_SLIP)");
    if (!isfinite(q.le_u)) return bad("le_u must be finite");
    if (q.le_u != 0.0 && (q.flags & MPC_WALLS_Z))
      return bad("le_u (Lees-Edwards) needs a periodic box (no MPC_WALLS_Z)");
    if ((q.flags & MPC_AMC) && (q.flags & MPC_WALLS_Z) && !(q.flags & MPC_SLIP))
      return bad("MPC_AMC is defined for periodic boxes and slip walls (MPC_SLIP)");
    if (q.form != p[0].form || q.flags != p[0].flags || q.reorder_every != p[0].reorder_every)
      return bad("form, flags and reorder_every must be equal for all boxes");
    if (q.reorder_every < 0) return bad("reorder_every < 0");
    for (int k = 0; k < 3; ++k)
      if (q.L[k] < 1) return bad("L must be >= 1");
    if (!(q.a > 0.0) || !isfinite(q.a)) return bad("a must be > 0");
    if (!(q.density > 0.0) || !isfinite(q.density)) return bad("density must be > 0");
    if (!(q.dt > 0.0) || !isfinite(q.dt)) return bad("dt must be > 0");
    if (!isfinite(q.alpha)) return bad("alpha must be finite");
    if (!(q.kT > 0.0) || !isfinite(q.kT)) return bad("kT must be > 0");
    if (!(q.mass > 0.0) || !isfinite(q.mass)) return bad("mass must be > 0");
    for (int k = 0; k < 3; ++k)
      if (!isfinite(q.g[k])) return bad("g must be finite");
    if (q.form == MPC_SPLIT32) {
      const int zmax = (q.flags & MPC_WALLS_Z) ? 1023 : 1024;
      if (q.L[0] > 2048 || q.L[1] > 2048 || q.L[2] > zmax) {
        snprintf(msg, sizeof msg, "box %d: split form needs L0, L1 <= 2048, L2 <= %d", b, zmax);
        *why = msg;
        return MPC_ERANGE;
      }
    }
  }
  return MPC_OK;
}

int make_plan(const mpc_params* p, int32_t nbox, Plan& P, std::string* why) {
  int rc = validate(p, nbox, why);
  if (rc) return rc;
  P.box.resize(nbox);
  for (int32_t b = 0; b < nbox; ++b) {
    const mpc_params& q = p[b];
    const bool walls = q.flags & MPC_WALLS_Z;
    const double vol = (double)q.L[0] * q.L[1] * q.L[2];
    const double nd = llround(q.density * vol);
    const int nlz = walls ? q.L[2] + 2 : q.L[2];
    const double cd = (double)q.L[0] * q.L[1] * nlz;
    if (nd < 1.0) {
      *why = "box with no particles";
      return MPC_EINVAL;
    }
    if (nd > (double)kMaxIndex || cd > (double)kMaxIndex) {
      *why = "particles or cells of a box >= 2^31";
      return MPC_ERANGE;
    }
    P.box[b].n = (uint64_t)nd;
    P.box[b].ncell = (uint64_t)cd;
    P.box[b].nlz = nlz;
    P.ntot += P.box[b].n;
    P.ctot += P.box[b].ncell;
    P.max_tiles += (uint64_t)q.L[1] * nlz * ((q.L[0] + kMinTileCells - 1) / kMinTileCells);
    P.npblocks += (P.box[b].n + kPartBlock - 1) / kPartBlock;
  }
  P.nscan = (uint32_t)((P.ctot + kScanBlock - 1) / kScanBlock);
  P.cpad = (uint64_t)P.nscan * kScanBlock;
  if (P.ntot > kMaxIndex || P.cpad + 1 > kMaxIndex) {
    *why = "total particles or cells >= 2^31";
    return MPC_ERANGE;
  }
  const int form = p[0].form;
  P.split = form == MPC_SPLIT32;
  P.rec = form == MPC_FP64 ? sizeof(RecF64) : (form == MPC_FP32 ? sizeof(RecF32) : sizeof(RecSplit));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  for (int s = 0; s < 2; ++s) {
    P.off_rec[s] = take(P.rec * P.ntot);
    P.off_id[s] = P.split ? 0 : take(4 * P.ntot);
  }
  P.off_key = take(4 * P.ntot);
  P.off_perm = take(4 * P.ntot);
  P.off_rank = take(2 * P.ntot);
  P.off_hist = take(4 * P.cpad);
  P.off_offset = take(4 * (P.cpad + 1));
  P.off_scan = take(4 * (size_t)P.nscan);
  P.off_ctrl = take(sizeof(Ctrl));
  P.off_boxes = take(sizeof(BoxDev) * nbox);
  P.off_tiles = take(sizeof(Tile) * P.max_tiles);
  P.off_pblocks = take(sizeof(PBlock) * P.npblocks);
  P.off_partials = take(sizeof(double) * 4 * P.npblocks);
  P.off_vmean = take(sizeof(double) * 3 * nbox);
  P.off_draws = take(sizeof(CellDraw) * P.cpad);
  P.off_phs = (p[0].flags & MPC_WALLS_Z) ? take(sizeof(PhantomSums) * P.cpad) : 0;
  P.total = off;
  return MPC_OK;
}

// Device scratch of the allocation-free entry point: the whole workspace of
// one call lives here.  Each device holds its own copy from module load to
// process end; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MPC_EHIP;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return MPC_EHIP;
    scratch_ptr[dev] = ptr;
  }
  *out = scratch_ptr[dev];
  return MPC_OK;
}

struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) {
      c += (s - t) + x;
    } else {
      c += (x - t) + s;
    }
    s = t;
  }
  double val() const { return s + c; }
};

}  // namespace

struct mpc_sim {
  std::vector<mpc_params> params;
  Plan plan;
  std::vector<BoxDev> boxes;
  std::vector<Tile> tiles;
  std::vector<PBlock> pblocks;
  std::vector<uint32_t> box_pb0;  // first pblock of each box, nbox + 1 entries
  Dev dev{};
  Launch L{};
  int form = 0;
  int32_t R = 0;
  uint64_t step = 0;
  uint32_t cur = 0;
  bool keys_valid = false;
  bool have_binning = false;
  bool use_graph = true;
  int32_t graph_steps = 1;         // steps per replay of the chunk graph
  bool graph_ready = false;
  hipGraphExec_t gexec = nullptr;  // one step
  hipGraphExec_t gexec_k = nullptr;  // graph_steps steps (graph_steps > 1)
  hipStream_t capture_stream = nullptr;
  int tile_override = 0, grid_override = 0, yblock = 8;
  int order = 0;  // tile order: 0 = row by row inside a block of rows, 1 = x-segment major
  int num_cu = 256, occupancy = 4;
  double* vmean = nullptr;
  std::string err;
};

namespace {

int hip_fail(mpc_sim* s, hipError_t e, const char* where) {
  if (e == hipSuccess) return MPC_OK;
  if (s) {
    s->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return MPC_EHIP;
}
#define HIPCHK(s, expr)                                  \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hip_fail((s), _e, #expr); \
  } while (0)

// Cells per tile so that a tile's mean particle count is ~95 % of the LDS
// capacity of one pass (larger tiles amortise the per-tile work; the Poisson
// excess of a full tile goes to a second pass).
int auto_tile_cells(double density) {
  const double target = 0.95 * kTileCap / density;
  return (int)std::max<double>(kMinTileCells, std::min<double>(kTileMaxCells, floor(target)));
}

// Tiles are runs of at most T consecutive cells inside one row (fixed y and z),
// so a tile's particles land in the rows y +- 1, z +- 1 of the next step and
// its next-step histogram fits a small on-chip window.  Tiles are listed so
// that the persistent grid, which hands each XCD a contiguous part of the list,
// keeps cells that exchange particles on one XCD at the same time: each XCD
// gets a slab of z planes, walked in blocks of `yblock` rows with z inside a
// block (order 0: each row's tiles in turn; order 1: one x segment of all
// rows of the block, then the next), so the rows a tile reads from are in
// flight together.
void build_tiles(mpc_sim* s) {
  s->tiles.clear();
  struct Keyed {
    uint64_t k;
    Tile t;
  };
  std::vector<Keyed> keyed;
  const int yb = std::max(1, s->yblock);
  for (size_t b = 0; b < s->boxes.size(); ++b) {
    const BoxDev& B = s->boxes[b];
    int T = s->tile_override ? s->tile_override : auto_tile_cells(B.density);
    T = std::max(kMinTileCells, std::min(kTileMaxCells, T));
    const uint64_t L0 = (uint64_t)B.L[0], L1 = (uint64_t)B.L[1];
    for (uint64_t cz = 0; cz < (uint64_t)B.nlz; ++cz) {
      for (uint64_t cy = 0; cy < L1; ++cy) {
        for (uint64_t cx = 0; cx < L0; cx += T) {
          Tile t;
          t.c0 = B.cbase + (uint32_t)((cz * L1 + cy) * L0 + cx);
          t.nc = (uint16_t)std::min<uint64_t>(T, L0 - cx);
          t.box = (uint16_t)b;
          t.x0 = (uint32_t)cx;
          t.y0 = (uint32_t)cy;
          t.z0 = (uint32_t)cz;
          const uint64_t slab = cz * 8 / (uint64_t)B.nlz;
          const uint64_t head = ((uint64_t)b * 8 + slab) << 12 | (cy / yb);
          // order 0: the rows of a block one after the other; order 1: the
          // same x segment of every row of the block, then the next segment
          // (the rows that exchange particles are in flight together)
          const uint64_t k =
              s->order == 0 ? (((head << 11 | cz) << 11 | cy) << 12) | (cx & 0xfff)
                            : (((head << 12 | (cx / (uint64_t)T)) << 11 | cz) << 11) | cy;
          keyed.push_back({k, t});
        }
      }
    }
  }
  std::stable_sort(keyed.begin(), keyed.end(),
                   [](const Keyed& a, const Keyed& b) { return a.k < b.k; });
  for (const Keyed& kt : keyed) s->tiles.push_back(kt.t);
  s->L.ntiles = (uint32_t)s->tiles.size();
  // default persistent grid: at most 8 one-wave workgroups per CU in flight
  // (more waves per XCD evict the gathered rows from L2), oversubscribed 2x
  // so that freed slots take the remaining workgroups (tail balance)
  uint32_t g = s->grid_override ? (uint32_t)s->grid_override
                                : (uint32_t)(2 * s->num_cu * std::min(8, std::max(1, s->occupancy)));
  g = std::max<uint32_t>(1, std::min<uint32_t>(g, s->L.ntiles));
  s->L.collide_grid = g;
}

int upload_tables(mpc_sim* s) {
  HIPCHK(s, hipMemcpyAsync(s->dev.tiles, s->tiles.data(), sizeof(Tile) * s->tiles.size(),
                           hipMemcpyHostToDevice, s->L.stream));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  return MPC_OK;
}

int read_ctrl(mpc_sim* s, Ctrl* c) {
  HIPCHK(s, hipMemcpyAsync(c, s->dev.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->L.stream));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  return MPC_OK;
}

int check_sticky(mpc_sim* s) {
  Ctrl c;
  int rc = read_ctrl(s, &c);
  if (rc) return rc;
  if (c.err & kErrKey) {
    s->err = "a particle left the box or is not finite";
    return MPC_ESTATE;
  }
  if (c.err & kErrCellOverflow) {
    s->err = "a collision cell held more than MPC_MAX_CELL_PARTICLES (256) particles; "
             "it was streamed but not collided";
    return MPC_ERANGE;
  }
  if (c.err & kErrFixRange) {
    s->err = "a fixed-point summand was outside |x| < 2^37 (cell units)";
    return MPC_ERANGE;
  }
  return MPC_OK;
}

// One step's launches (scan, scatter, collide, advance) on `st`.
hipError_t enqueue_step(mpc_sim* s, hipStream_t st) {
  Launch l = s->L;
  l.stream = st;
  hipError_t e;
  if ((e = launch_scan(s->dev, l)) != hipSuccess) return e;
  if ((e = launch_phantoms(s->dev, l)) != hipSuccess) return e;
  if ((e = launch_scatter(s->dev, l)) != hipSuccess) return e;
  if ((e = launch_collide(s->dev, l)) != hipSuccess) return e;
  return launch_advance(s->dev, l);
}

int ensure_keys(mpc_sim* s) {
  if (s->keys_valid) return MPC_OK;
  HIPCHK(s, launch_zero_u32(s->dev.hist, s->plan.cpad, s->L.stream));
  HIPCHK(s, launch_key_hist(s->dev, s->L));
  s->keys_valid = true;
  return MPC_OK;
}

void advance_mirror(mpc_sim* s, int64_t n) {
  s->cur ^= (uint32_t)(n & 1);
  s->step += (uint64_t)n;
}

int drop_graph(mpc_sim* s) {
  if (s->gexec) {
    HIPCHK(s, hipGraphExecDestroy(s->gexec));
    s->gexec = nullptr;
  }
  if (s->gexec_k) {
    HIPCHK(s, hipGraphExecDestroy(s->gexec_k));
    s->gexec_k = nullptr;
  }
  s->graph_ready = false;
  return MPC_OK;
}

// One executable graph of `steps` consecutive steps (every step reads the
// step counter and the state buffer index from device memory, so one graph
// serves every replay).
int capture_steps(mpc_sim* s, int32_t steps, hipGraphExec_t* out) {
  if (!s->capture_stream) HIPCHK(s, hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHK(s, hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int32_t k = 0; k < steps && e == hipSuccess; ++k) e = enqueue_step(s, s->capture_stream);
  hipError_t e2 = hipStreamEndCapture(s->capture_stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(s, e, "capture step");
  }
  if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamEndCapture");
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
  return MPC_OK;
}

int capture_graph(mpc_sim* s) {
  if (s->graph_ready) return MPC_OK;
  int rc = capture_steps(s, 1, &s->gexec);
  if (!rc && s->graph_steps > 1) rc = capture_steps(s, s->graph_steps, &s->gexec_k);
  if (rc) return rc;
  s->graph_ready = true;
  return MPC_OK;
}

// Host FP64 <-> stored form of one box.
template <typename T>
int copy_h2d(mpc_sim* s, void* dst_base, uint64_t elem0, const std::vector<T>& src) {
  HIPCHK(s, hipMemcpyAsync((T*)dst_base + elem0, src.data(), sizeof(T) * src.size(),
                           hipMemcpyHostToDevice, s->L.stream));
  return MPC_OK;
}
template <typename T>
int copy_d2h(mpc_sim* s, const void* src_base, uint64_t elem0, std::vector<T>& dst) {
  HIPCHK(s, hipMemcpyAsync(dst.data(), (const T*)src_base + elem0, sizeof(T) * dst.size(),
                           hipMemcpyDeviceToHost, s->L.stream));
  return MPC_OK;
}

// Logical indices of slots p0 .. p0 + out.size() - 1 of state buffer S: a copy
// of the id array, or of the records a chunk at a time (ids inside records).
int read_ids(mpc_sim* s, const StatePtrs& S, uint64_t p0, std::vector<uint32_t>& out) {
  const uint64_t n = out.size();
  if (S.id_stride == 1) {
    HIPCHK(s, hipMemcpyAsync(out.data(), S.id + p0, sizeof(uint32_t) * n, hipMemcpyDeviceToHost,
                             s->L.stream));
    HIPCHK(s, hipStreamSynchronize(s->L.stream));
    return MPC_OK;
  }
  const uint64_t st = S.id_stride;
  const uint64_t w = (uint64_t)(S.id - (const uint32_t*)S.rec);  // id word inside a record
  const uint64_t chunk = std::min<uint64_t>(n, (uint64_t)kStateChunk);
  std::vector<uint32_t> buf((size_t)(chunk * st));
  for (uint64_t i0 = 0; i0 < n; i0 += chunk) {
    const uint64_t m = std::min(chunk, n - i0);
    HIPCHK(s, hipMemcpyAsync(buf.data(), (const uint32_t*)S.rec + (p0 + i0) * st,
                             sizeof(uint32_t) * m * st, hipMemcpyDeviceToHost, s->L.stream));
    HIPCHK(s, hipStreamSynchronize(s->L.stream));
    for (uint64_t i = 0; i < m; ++i) out[i0 + i] = buf[i * st + w];
  }
  return MPC_OK;
}

int obs_all(mpc_sim* s, std::vector<double>& P, std::vector<double>& E,
            std::vector<double>& K) {
  const size_t nbox = s->boxes.size();
  const size_t npb = s->pblocks.size();
  std::vector<double> part(4 * npb);
  HIPCHK(s, launch_obs_pass1(s->dev, s->L));
  HIPCHK(s, hipMemcpyAsync(part.data(), s->dev.partials, sizeof(double) * 4 * npb,
                           hipMemcpyDeviceToHost, s->L.stream));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  P.assign(3 * nbox, 0.0);
  E.assign(nbox, 0.0);
  K.assign(nbox, 0.0);
  std::vector<double> vm(3 * nbox);
  for (size_t b = 0; b < nbox; ++b) {
    Neumaier a[4];
    for (uint32_t q = s->box_pb0[b]; q < s->box_pb0[b + 1]; ++q)
      for (int k = 0; k < 4; ++k) a[k].add(part[4 * q + k]);
    for (int k = 0; k < 3; ++k) P[3 * b + k] = a[k].val();
    E[b] = a[3].val();
    const double M = (double)s->boxes[b].np * s->boxes[b].mass;
    for (int k = 0; k < 3; ++k) vm[3 * b + k] = P[3 * b + k] / M;
  }
  HIPCHK(s, hipMemcpyAsync(s->vmean, vm.data(), sizeof(double) * 3 * nbox, hipMemcpyHostToDevice,
                           s->L.stream));
  HIPCHK(s, launch_obs_pass2(s->dev, s->L, s->vmean));
  HIPCHK(s, hipMemcpyAsync(part.data(), s->dev.partials, sizeof(double) * 4 * npb,
                           hipMemcpyDeviceToHost, s->L.stream));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  for (size_t b = 0; b < nbox; ++b) {
    Neumaier a;
    for (uint32_t q = s->box_pb0[b]; q < s->box_pb0[b + 1]; ++q) a.add(part[4 * q]);
    K[b] = a.val();
  }
  return MPC_OK;
}

}  // namespace

extern "C" {

const char* mpc_strerror(int code) {
  switch (code) {
    case MPC_OK: return "ok";
    case MPC_EINVAL: return "invalid argument";
    case MPC_ENOSPACE: return "workspace too small";
    case MPC_ERANGE: return "size out of range";
    case MPC_EHIP: return "HIP runtime error";
    case MPC_ESTATE: return "invalid particle state";
    default: return "unknown error";
  }
}

const char* mpc_last_error(mpc_sim* s) { return s ? s->err.c_str() : ""; }

int mpc_workspace_bytes(const mpc_params* p, int32_t nbox, size_t* bytes) {
  if (!bytes) return MPC_EINVAL;
  Plan P;
  std::string why;
  const int rc = make_plan(p, nbox, P, &why);
  if (rc) return rc;
  *bytes = P.total;
  return MPC_OK;
}

int mpc_create(const mpc_params* p, int32_t nbox, void* workspace, size_t bytes,
               void* hip_stream, mpc_sim** out) {
  if (!out) return MPC_EINVAL;
  *out = nullptr;
  mpc_sim* s = new mpc_sim();
  std::string why;
  int rc = make_plan(p, nbox, s->plan, &why);
  if (rc) {
    delete s;
    return rc;
  }
  if (!workspace || bytes < s->plan.total || ((uintptr_t)workspace & 255)) {
    delete s;
    return workspace && bytes >= s->plan.total ? MPC_EINVAL : MPC_ENOSPACE;
  }
  s->params.assign(p, p + nbox);
  s->form = p[0].form;
  s->R = p[0].reorder_every;
  const Plan& P = s->plan;
  char* ws = (char*)workspace;
  for (int b = 0; b < 2; ++b) {
    s->dev.S[b].rec = ws + P.off_rec[b];
    s->dev.S[b].id = P.split ? &((RecSplit*)(ws + P.off_rec[b]))->id : (uint32_t*)(ws + P.off_id[b]);
    s->dev.S[b].id_stride = P.split ? (uint32_t)(sizeof(RecSplit) / 4) : 1u;
  }
  s->dev.key = (uint32_t*)(ws + P.off_key);
  s->dev.perm = (uint32_t*)(ws + P.off_perm);
  s->dev.rank = (uint16_t*)(ws + P.off_rank);
  s->dev.hist = (uint32_t*)(ws + P.off_hist);
  s->dev.offset = (uint32_t*)(ws + P.off_offset);
  s->dev.scan_blk = (uint32_t*)(ws + P.off_scan);
  s->dev.ctrl = (Ctrl*)(ws + P.off_ctrl);
  s->dev.boxes = (BoxDev*)(ws + P.off_boxes);
  s->dev.tiles = (Tile*)(ws + P.off_tiles);
  s->dev.pblocks = (PBlock*)(ws + P.off_pblocks);
  s->dev.partials = (double*)(ws + P.off_partials);
  s->dev.ntot = (uint32_t)P.ntot;
  s->vmean = (double*)(ws + P.off_vmean);
  s->dev.draws = (CellDraw*)(ws + P.off_draws);
  s->dev.phs = (p[0].flags & MPC_WALLS_Z) ? (PhantomSums*)(ws + P.off_phs) : nullptr;

  // boxes
  uint64_t pb = 0, cb = 0, wcb = 0;
  s->box_pb0.push_back(0);
  for (int32_t b = 0; b < nbox; ++b) {
    const mpc_params& q = p[b];
    BoxDev B{};
    for (int k = 0; k < 3; ++k) {
      B.L[k] = q.L[k];
      B.Ld[k] = (double)q.L[k];
      B.Lf[k] = (float)q.L[k];
    }
    B.nlz = P.box[b].nlz;
    B.pbase = (uint32_t)pb;
    B.np = (uint32_t)P.box[b].n;
    B.cbase = (uint32_t)cb;
    B.nc = (uint32_t)P.box[b].ncell;
    B.key_lo = (uint32_t)(q.seed & 0xffffffffu);
    B.key_hi = (uint32_t)(q.seed >> 32);
    B.walls = (q.flags & MPC_WALLS_Z) ? 1u : 0u;
    B.mbs = (q.flags & MPC_MBS) ? 1u : 0u;
    // internal units: lengths in cells, so velocities / a, energies / a^2
    B.h = q.dt;
    B.hf = (float)q.dt;
    B.ca = cos(q.alpha);
    B.sa = sin(q.alpha);
    B.omc = 1.0 - B.ca;
    B.kT = q.kT / (q.a * q.a);
    B.mass = q.mass;
    B.density = q.density;
    B.sd = sqrt(B.kT / q.mass);
    B.grav = (q.g[0] != 0.0 || q.g[1] != 0.0 || q.g[2] != 0.0) ? 1u : 0u;
    B.wcbase = (uint32_t)wcb;
    if (B.walls) wcb += 2ull * (uint64_t)q.L[0] * (uint64_t)q.L[1];
    for (int k = 0; k < 3; ++k) B.gh[k] = (q.g[k] / q.a) * q.dt;
    B.slip = (B.walls && (q.flags & MPC_SLIP)) ? 1u : 0u;
    B.uw = q.wall_u / q.a;
    B.uwf = (float)B.uw;
    B.le = (!B.walls && q.le_u != 0.0) ? 1u : 0u;
    if (B.le) s->L.le = 1;
    B.leu = q.le_u / q.a;
    B.leuf = (float)B.leu;
    s->boxes.push_back(B);
    for (uint64_t p0 = 0; p0 < P.box[b].n; p0 += kPartBlock)
      s->pblocks.push_back(PBlock{(uint32_t)b, (uint32_t)(pb + p0)});
    s->box_pb0.push_back((uint32_t)s->pblocks.size());
    pb += P.box[b].n;
    cb += P.box[b].ncell;
  }

  s->L.form = s->form;
  s->L.round_phantoms = s->form == MPC_SPLIT32 ? 1 : 0;
  s->L.wcells = (uint32_t)wcb;
  s->L.walls = (p[0].flags & MPC_WALLS_Z) ? 1 : 0;
  s->L.mbs = (p[0].flags & MPC_MBS) ? 1 : 0;
  s->L.amc = (p[0].flags & MPC_AMC) ? 1 : 0;
  s->L.fixed = (p[0].flags & MPC_FIXED_SUMS) ? 1 : 0;
  s->L.nbox = (uint32_t)nbox;
  s->L.ntot = P.ntot;
  s->L.ctot = P.ctot;
  s->L.nscan = P.nscan;
  s->L.npblocks = (uint32_t)s->pblocks.size();
  s->L.stream = (hipStream_t)hip_stream;
  s->L.xcd_remap = 1;

  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    s->num_cu = prop.multiProcessorCount;
  s->occupancy = 2;
  if (collide_occupancy(s->L, &s->occupancy) != hipSuccess ||
      s->occupancy < 1)
    s->occupancy = 1;
  build_tiles(s);

  auto fail = [&](int code) {
    delete s;
    return code;
  };
  if ((rc = upload_tables(s))) return fail(rc);
  if (hipMemcpyAsync(s->dev.boxes, s->boxes.data(), sizeof(BoxDev) * s->boxes.size(),
                     hipMemcpyHostToDevice, s->L.stream) != hipSuccess ||
      hipMemcpyAsync(s->dev.pblocks, s->pblocks.data(), sizeof(PBlock) * s->pblocks.size(),
                     hipMemcpyHostToDevice, s->L.stream) != hipSuccess ||
      launch_zero_u32(s->dev.hist, P.cpad, s->L.stream) != hipSuccess ||
      launch_zero_u32(s->dev.perm, P.ntot, s->L.stream) != hipSuccess ||
      launch_zero_u32(s->dev.key, P.ntot, s->L.stream) != hipSuccess ||
      launch_zero_u32((uint32_t*)s->dev.rank, (P.ntot + 1) / 2, s->L.stream) != hipSuccess ||
      launch_zero_u32(s->dev.offset, P.cpad + 1, s->L.stream) != hipSuccess ||
      launch_set_ctrl(s->dev, s->L, 0, 0, s->R, 1) != hipSuccess ||
      hipStreamSynchronize(s->L.stream) != hipSuccess)
    return fail(MPC_EHIP);
  *out = s;
  return MPC_OK;
}

int mpc_destroy(mpc_sim* s) {
  if (!s) return MPC_EINVAL;
  (void)hipStreamSynchronize(s->L.stream);
  drop_graph(s);
  if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
  delete s;
  return MPC_OK;
}

int mpc_set_graph(mpc_sim* s, int32_t enable) {
  if (!s || enable < 0 || enable > kMaxGraphSteps) return MPC_EINVAL;
  if (enable >= 1 && enable != s->graph_steps) {
    HIPCHK(s, hipStreamSynchronize(s->L.stream));
    int rc = drop_graph(s);
    if (rc) return rc;
    s->graph_steps = enable;
  }
  s->use_graph = enable != 0;
  return MPC_OK;
}

int mpc_set_tiling(mpc_sim* s, int32_t tile_cells, int32_t grid, int32_t yblock,
                   int32_t order) {
  if (!s) return MPC_EINVAL;
  if (tile_cells != 0 && (tile_cells < kMinTileCells || tile_cells > kTileMaxCells))
    return MPC_EINVAL;
  if (grid < 0 || yblock < 0 || yblock > 4096 || order < 0 || order > 1) return MPC_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  s->tile_override = tile_cells;
  s->grid_override = grid;
  s->yblock = yblock ? yblock : 8;
  s->order = order;
  build_tiles(s);
  int rc = drop_graph(s);
  if (rc) return rc;
  return upload_tables(s);
}

int mpc_get_tiling(mpc_sim* s, int32_t* tile_cells, int32_t* grid, int32_t* yblock,
                   int32_t* order, int64_t* ntiles) {
  if (!s) return MPC_EINVAL;
  if (tile_cells) *tile_cells = s->tile_override;
  if (grid) *grid = (int32_t)s->L.collide_grid;
  if (yblock) *yblock = s->yblock;
  if (order) *order = s->order;
  if (ntiles) *ntiles = (int64_t)s->L.ntiles;
  return MPC_OK;
}

int mpc_step(mpc_sim* s, int64_t nsteps) {
  if (!s || nsteps < 0) return MPC_EINVAL;
  if (nsteps == 0) return MPC_OK;
  int rc = ensure_keys(s);
  if (rc) return rc;
  if (s->use_graph) {
    if ((rc = capture_graph(s))) return rc;
    int64_t k = 0;
    if (s->gexec_k)
      for (; k + s->graph_steps <= nsteps; k += s->graph_steps)
        HIPCHK(s, hipGraphLaunch(s->gexec_k, s->L.stream));
    for (; k < nsteps; ++k) HIPCHK(s, hipGraphLaunch(s->gexec, s->L.stream));
  } else {
    for (int64_t k = 0; k < nsteps; ++k) HIPCHK(s, enqueue_step(s, s->L.stream));
  }
  advance_mirror(s, nsteps);
  s->have_binning = true;
  return MPC_OK;
}

int mpc_step_profiled(mpc_sim* s, int64_t nsteps, mpc_kernel_times* acc) {
  if (!s || nsteps < 0 || !acc) return MPC_EINVAL;
  if (nsteps == 0) return MPC_OK;
  hipStream_t st = s->L.stream;
  std::vector<hipEvent_t> ev;
  auto mark = [&]() -> hipError_t {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
    return hipEventRecord(e, st);
  };
  int kinds_prologue = 0;
  HIPCHK(s, mark());
  if (!s->keys_valid) {
    HIPCHK(s, launch_zero_u32(s->dev.hist, s->plan.cpad, st));
    HIPCHK(s, launch_key_hist(s->dev, s->L));
    s->keys_valid = true;
    HIPCHK(s, mark());
    kinds_prologue = 1;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    HIPCHK(s, launch_scan(s->dev, s->L));
    HIPCHK(s, launch_phantoms(s->dev, s->L));
    HIPCHK(s, mark());
    HIPCHK(s, launch_scatter(s->dev, s->L));
    HIPCHK(s, mark());
    HIPCHK(s, launch_collide(s->dev, s->L));
    HIPCHK(s, mark());
    HIPCHK(s, launch_advance(s->dev, s->L));
    HIPCHK(s, mark());
  }
  HIPCHK(s, hipStreamSynchronize(st));
  size_t e = 0;
  auto span = [&]() {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[e], ev[e + 1]);
    ++e;
    return (double)ms;
  };
  if (kinds_prologue) {
    acc->prologue_ms += span();
    acc->prologue_launches += 1;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    acc->scan_ms += span();
    acc->scatter_ms += span();
    acc->collide_ms += span();
    acc->other_ms += span();
    acc->scan_launches += 1;
    acc->scatter_launches += 1;
    acc->collide_launches += 1;
  }
  for (hipEvent_t x : ev) (void)hipEventDestroy(x);
  advance_mirror(s, nsteps);
  s->have_binning = true;
  return MPC_OK;
}

int mpc_sync(mpc_sim* s) {
  if (!s) return MPC_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  return check_sticky(s);
}

int mpc_box_info(mpc_sim* s, int32_t box, int64_t* n, int64_t* ncell) {
  if (!s || box < 0 || box >= (int32_t)s->boxes.size()) return MPC_EINVAL;
  if (n) *n = (int64_t)s->boxes[box].np;
  if (ncell) *ncell = (int64_t)s->boxes[box].nc;
  return MPC_OK;
}

int mpc_get_step(mpc_sim* s, uint64_t* step) {
  if (!s || !step) return MPC_EINVAL;
  *step = s->step;
  return MPC_OK;
}

int mpc_set_step(mpc_sim* s, uint64_t step) {
  if (!s) return MPC_EINVAL;
  s->step = step;
  s->keys_valid = false;
  s->have_binning = false;
  HIPCHK(s, launch_set_ctrl(s->dev, s->L, s->step, s->cur, s->R, 0));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  return MPC_OK;
}

int mpc_init_state(mpc_sim* s, uint64_t init_seed) {
  if (!s) return MPC_EINVAL;
  HIPCHK(s, launch_set_ctrl(s->dev, s->L, s->step, s->cur, s->R, 1));
  HIPCHK(s, launch_init_state(s->dev, s->L, init_seed));
  std::vector<double> P, E, K;
  // mean of each box
  const size_t nbox = s->boxes.size();
  const size_t npb = s->pblocks.size();
  std::vector<double> part(4 * npb);
  HIPCHK(s, launch_obs_pass1(s->dev, s->L));
  HIPCHK(s, hipMemcpyAsync(part.data(), s->dev.partials, sizeof(double) * 4 * npb,
                           hipMemcpyDeviceToHost, s->L.stream));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  std::vector<double> vm(3 * nbox);
  for (size_t b = 0; b < nbox; ++b) {
    Neumaier a[3];
    for (uint32_t q = s->box_pb0[b]; q < s->box_pb0[b + 1]; ++q)
      for (int k = 0; k < 3; ++k) a[k].add(part[4 * q + k]);
    const double M = (double)s->boxes[b].np * s->boxes[b].mass;
    for (int k = 0; k < 3; ++k) vm[3 * b + k] = a[k].val() / M;
  }
  HIPCHK(s, hipMemcpyAsync(s->vmean, vm.data(), sizeof(double) * 3 * nbox, hipMemcpyHostToDevice,
                           s->L.stream));
  HIPCHK(s, launch_remove_mean(s->dev, s->L, s->vmean));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  s->keys_valid = false;
  s->have_binning = false;
  return MPC_OK;
}

int mpc_set_state(mpc_sim* s, int32_t box, const double* x, const double* v, int64_t n) {
  if (!s || box < 0 || box >= (int32_t)s->boxes.size() || !x || !v) return MPC_EINVAL;
  const BoxDev& B = s->boxes[box];
  if (n != (int64_t)B.np) {
    s->err = "n differs from the box's particle count";
    return MPC_EINVAL;
  }
  const double a = s->params[box].a;
  const bool walls = B.walls;
  // validate positions (internal units)
  for (int k = 0; k < 3; ++k) {
    const double Lk = B.Ld[k];
    for (int64_t i = 0; i < n; ++i) {
      const double xi = x[k * n + i] / a;
      const bool ok = (walls && k == 2) ? (xi >= 0.0 && xi <= Lk) : (xi >= 0.0 && xi < Lk);
      if (!ok || !isfinite(v[k * n + i])) {
        s->err = "position outside the box or non-finite velocity";
        return MPC_EINVAL;
      }
    }
  }
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  // records (and ids) of the box, packed on the host a chunk at a time
  const StatePtrs& S = s->dev.S[s->cur];
  const size_t rb = s->plan.rec;
  const int64_t chunk = std::min<int64_t>(n, kStateChunk);
  std::vector<unsigned char> rbuf((size_t)chunk * rb);
  std::vector<uint32_t> ibuf(s->plan.split ? 0 : (size_t)chunk);
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    const int64_t m = std::min(chunk, n - i0);
    for (int64_t i = 0; i < m; ++i) {
      const int64_t g = i0 + i;
      const uint32_t id = B.pbase + (uint32_t)g;
      if (s->form == MPC_FP64) {
        RecF64& r = ((RecF64*)rbuf.data())[i];
        for (int k = 0; k < 3; ++k) {
          r.x[k] = x[k * n + g] / a;
          r.v[k] = v[k * n + g] / a;
        }
        ibuf[i] = id;
      } else if (s->form == MPC_FP32) {
        RecF32& r = ((RecF32*)rbuf.data())[i];
        for (int k = 0; k < 3; ++k) {
          float f = (float)(x[k * n + g] / a);
          if (!(walls && k == 2) && f >= B.Lf[k]) f = nextafterf(B.Lf[k], 0.0f);
          r.x[k] = f;
          r.v[k] = (float)(v[k * n + g] / a);
        }
        ibuf[i] = id;
      } else {
        RecSplit& r = ((RecSplit*)rbuf.data())[i];
        r.cell = 0u;
        for (int k = 0; k < 3; ++k) {
          const uint32_t shift = k == 0 ? 0 : (k == 1 ? kSplitXBits : kSplitXBits + kSplitYBits);
          const double xi = x[k * n + g] / a;
          double fl = floor(xi);
          float o = (float)(xi - fl);
          if (o >= 1.0f) {
            o = 0.0f;
            fl += 1.0;
          }
          int c = (int)fl;
          if (!(walls && k == 2) && c >= B.L[k]) c -= B.L[k];
          r.cell |= (uint32_t)c << shift;
          r.o[k] = o;
          r.v[k] = (float)(v[k * n + g] / a);
        }
        r.id = id;
      }
    }
    HIPCHK(s, hipMemcpyAsync((char*)S.rec + (B.pbase + (uint64_t)i0) * rb, rbuf.data(),
                             (size_t)m * rb, hipMemcpyHostToDevice, s->L.stream));
    if (!s->plan.split)
      HIPCHK(s, hipMemcpyAsync(S.id + B.pbase + i0, ibuf.data(), sizeof(uint32_t) * (size_t)m,
                               hipMemcpyHostToDevice, s->L.stream));
    HIPCHK(s, hipStreamSynchronize(s->L.stream));  // the staging buffers are reused
  }
  HIPCHK(s, launch_set_ctrl(s->dev, s->L, s->step, s->cur, s->R, 1));
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  s->keys_valid = false;
  s->have_binning = false;
  return MPC_OK;
}

int mpc_get_state(mpc_sim* s, int32_t box, double* x, double* v, int64_t n) {
  if (!s || box < 0 || box >= (int32_t)s->boxes.size() || !x || !v) return MPC_EINVAL;
  const BoxDev& B = s->boxes[box];
  if (n != (int64_t)B.np) return MPC_EINVAL;
  int rc = mpc_sync(s);
  if (rc) return rc;
  const double a = s->params[box].a;
  const StatePtrs& S = s->dev.S[s->cur];
  // records (and ids) of the box, a chunk at a time, each written to the
  // caller's order given by its logical index
  const size_t rb = s->plan.rec;
  const int64_t chunk = std::min<int64_t>(n, kStateChunk);
  std::vector<unsigned char> rbuf((size_t)chunk * rb);
  std::vector<uint32_t> ibuf(s->plan.split ? 0 : (size_t)chunk);
  std::vector<uint8_t> seen(n, 0);
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    const int64_t m = std::min(chunk, n - i0);
    HIPCHK(s, hipMemcpyAsync(rbuf.data(), (const char*)S.rec + (B.pbase + (uint64_t)i0) * rb,
                             (size_t)m * rb, hipMemcpyDeviceToHost, s->L.stream));
    if (!s->plan.split)
      HIPCHK(s, hipMemcpyAsync(ibuf.data(), S.id + B.pbase + i0, sizeof(uint32_t) * (size_t)m,
                               hipMemcpyDeviceToHost, s->L.stream));
    HIPCHK(s, hipStreamSynchronize(s->L.stream));
    for (int64_t i = 0; i < m; ++i) {
      const uint32_t id = s->plan.split ? ((const RecSplit*)rbuf.data())[i].id : ibuf[i];
      const uint32_t q = id - B.pbase;
      if (id < B.pbase || q >= (uint64_t)n || seen[q]) {
        s->err = "logical particle indices are not a permutation";
        return MPC_ESTATE;
      }
      seen[q] = 1;
      if (s->form == MPC_FP64) {
        const RecF64& r = ((const RecF64*)rbuf.data())[i];
        for (int k = 0; k < 3; ++k) {
          x[k * n + q] = r.x[k] * a;
          v[k * n + q] = r.v[k] * a;
        }
      } else if (s->form == MPC_FP32) {
        const RecF32& r = ((const RecF32*)rbuf.data())[i];
        for (int k = 0; k < 3; ++k) {
          x[k * n + q] = (double)r.x[k] * a;
          v[k * n + q] = (double)r.v[k] * a;
        }
      } else {
        const RecSplit& r = ((const RecSplit*)rbuf.data())[i];
        for (int k = 0; k < 3; ++k) {
          const uint32_t shift = k == 0 ? 0 : (k == 1 ? kSplitXBits : kSplitXBits + kSplitYBits);
          const uint32_t mask = k == 2 ? ((1u << kSplitZBits) - 1) : ((1u << kSplitXBits) - 1);
          x[k * n + q] = ((double)((r.cell >> shift) & mask) + (double)r.o[k]) * a;
          v[k * n + q] = (double)r.v[k] * a;
        }
      }
    }
  }
  return MPC_OK;
}

int mpc_get_particles(mpc_sim* s, int32_t box, const int64_t* idx, int64_t m, double* x,
                      double* v) {
  if (!s || box < 0 || box >= (int32_t)s->boxes.size() || m < 0) return MPC_EINVAL;
  if (m > 0 && (!idx || !x || !v)) return MPC_EINVAL;
  const BoxDev& B = s->boxes[box];
  if (m > (int64_t)kMaxIndex) {
    s->err = "more than 2^31 - 1 particles requested";
    return MPC_EINVAL;
  }
  std::vector<uint32_t> lidx((size_t)m);
  for (int64_t k = 0; k < m; ++k) {
    if (idx[k] < 0 || idx[k] >= (int64_t)B.np) {
      s->err = "particle index outside the box";
      return MPC_EINVAL;
    }
    lidx[k] = (uint32_t)idx[k];
  }
  int rc = mpc_sync(s);
  if (rc || m == 0) return rc;
  const StatePtrs& S = s->dev.S[s->cur];
  uint32_t* dinv = nullptr;
  uint32_t* dl = nullptr;
  double* dout = nullptr;
  std::vector<double> out(6 * (size_t)m);
  hipError_t e = hipSuccess;
  const char* where = "";
  do {
    if (S.id) {
      where = "hipMalloc (inverse index)";
      if ((e = hipMalloc(&dinv, sizeof(uint32_t) * (size_t)B.np)) != hipSuccess) break;
      where = "hipMemsetAsync";
      if ((e = hipMemsetAsync(dinv, 0xff, sizeof(uint32_t) * (size_t)B.np, s->L.stream)) !=
          hipSuccess)
        break;
    }
    where = "hipMalloc (sample)";
    if ((e = hipMalloc(&dl, sizeof(uint32_t) * (size_t)m)) != hipSuccess) break;
    if ((e = hipMalloc(&dout, sizeof(double) * 6 * (size_t)m)) != hipSuccess) break;
    where = "copy of the sample indices";
    if ((e = hipMemcpyAsync(dl, lidx.data(), sizeof(uint32_t) * (size_t)m,
                            hipMemcpyHostToDevice, s->L.stream)) != hipSuccess)
      break;
    where = "gather kernels";
    if ((e = launch_gather_particles(s->dev, s->L, S, dinv, B.pbase, B.np, dl, (uint32_t)m,
                                     dout)) != hipSuccess)
      break;
    where = "copy of the sample";
    if ((e = hipMemcpyAsync(out.data(), dout, sizeof(double) * 6 * (size_t)m,
                            hipMemcpyDeviceToHost, s->L.stream)) != hipSuccess)
      break;
    where = "hipStreamSynchronize";
    e = hipStreamSynchronize(s->L.stream);
  } while (false);
  if (dinv) (void)hipFree(dinv);
  if (dl) (void)hipFree(dl);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return hip_fail(s, e, where);
  const double a = s->params[box].a;
  for (int64_t k = 0; k < m; ++k) {
    if (isnan(out[k])) {
      s->err = "logical particle indices are not a permutation";
      return MPC_ESTATE;
    }
    for (int c = 0; c < 3; ++c) {
      x[c * m + k] = out[(size_t)c * m + k] * a;
      v[c * m + k] = out[(size_t)(3 + c) * m + k] * a;
    }
  }
  return MPC_OK;
}

int mpc_observables(mpc_sim* s, int32_t box, mpc_obs* out) {
  if (!s || !out || box < 0 || box >= (int32_t)s->boxes.size()) return MPC_EINVAL;
  int rc = mpc_sync(s);
  if (rc) return rc;
  std::vector<double> P, E, K;
  if ((rc = obs_all(s, P, E, K))) return rc;
  const BoxDev& B = s->boxes[box];
  const double a = s->params[box].a;
  out->step = s->step;
  out->n = B.np;
  for (int k = 0; k < 3; ++k) out->P[k] = P[3 * box + k] * a;
  out->E = E[box] * a * a;
  out->T = B.np > 1 ? K[box] / (3.0 * (double)(B.np - 1)) * a * a : 0.0;
  out->mass_total = (double)B.np * B.mass;
  if (!isfinite(out->E) || !isfinite(out->P[0]) || !isfinite(out->P[1]) || !isfinite(out->P[2])) {
    s->err = "non-finite observables";
    return MPC_ESTATE;
  }
  return MPC_OK;
}

int mpc_get_binning(mpc_sim* s, int32_t box, uint32_t* key, uint32_t* perm, uint32_t* offset) {
  if (!s || box < 0 || box >= (int32_t)s->boxes.size()) return MPC_EINVAL;
  if (!s->have_binning) {
    s->err = "no step since the state was set";
    return MPC_EINVAL;
  }
  int rc = mpc_sync(s);
  if (rc) return rc;
  // the last step read the buffer that is not current; its ids give the
  // logical order before that step
  const StatePtrs& Sin = s->dev.S[s->cur ^ 1u];
  HIPCHK(s, launch_canon_perm(s->dev, s->L, Sin));
  const BoxDev& B = s->boxes[box];
  std::vector<uint32_t> off(B.nc + 1), pm(B.np), lid(B.np);
  if ((rc = copy_d2h(s, s->dev.offset, B.cbase, off))) return rc;
  if ((rc = copy_d2h(s, s->dev.perm, B.pbase, pm))) return rc;
  HIPCHK(s, hipStreamSynchronize(s->L.stream));
  if ((rc = read_ids(s, Sin, B.pbase, lid))) return rc;
  const uint32_t o0 = off[0];
  for (auto& o : off) o -= o0;
  for (auto& q : pm) {
    if (q < B.pbase || q - B.pbase >= B.np) {
      s->err = "permutation entry outside the box";
      return MPC_ESTATE;
    }
    q = lid[q - B.pbase] - B.pbase;
    if (q >= B.np) {
      s->err = "logical particle index outside the box";
      return MPC_ESTATE;
    }
  }
  if (offset) memcpy(offset, off.data(), sizeof(uint32_t) * off.size());
  if (perm) memcpy(perm, pm.data(), sizeof(uint32_t) * pm.size());
  if (key) {
    for (uint32_t c = 0; c < B.nc; ++c)
      for (uint32_t j = off[c]; j < off[c + 1]; ++j) key[pm[j]] = c;
  }
  return MPC_OK;
}

int mpc_autotune(mpc_sim* s, int32_t trial_steps, int32_t* tile_cells, int32_t* grid) {
  if (!s || trial_steps < 1 || trial_steps > 1000) return MPC_EINVAL;
  int rc = mpc_sync(s);
  if (rc) return rc;
  const Plan& P = s->plan;
  hipStream_t st = s->L.stream;
  const uint64_t step0 = s->step;
  const uint32_t cur0 = s->cur;
  const int T0 = s->tile_override, g0 = s->grid_override, y0 = s->yblock, o0 = s->order;
  // the arrays of the current state buffer, backed up on the device (or in
  // host memory if the device has no room) and restored before every trial
  std::vector<std::pair<void*, size_t>> arrs;
  const StatePtrs& S = s->dev.S[cur0];
  arrs.push_back({S.rec, P.rec * P.ntot});
  if (!P.split) arrs.push_back({S.id, 4 * P.ntot});
  size_t total = 0;
  for (auto& a : arrs) total += align256(a.second);
  void* backup = nullptr;
  bool on_host = false;
  if (hipMalloc(&backup, total) != hipSuccess) {
    (void)hipGetLastError();
    backup = nullptr;
    if (hipHostMalloc(&backup, total, hipHostMallocDefault) != hipSuccess) {
      s->err = "autotune: no memory for the state backup";
      return MPC_EHIP;
    }
    on_host = true;
  }
  auto copy_all = [&](bool save) -> hipError_t {
    size_t o = 0;
    for (auto& a : arrs) {
      char* bk = (char*)backup + o;
      hipError_t e = save ? hipMemcpyAsync(bk, a.first, a.second, hipMemcpyDefault, st)
                          : hipMemcpyAsync(a.first, bk, a.second, hipMemcpyDefault, st);
      if (e != hipSuccess) return e;
      o += align256(a.second);
    }
    return hipStreamSynchronize(st);
  };
  auto release = [&]() {
    if (on_host) {
      (void)hipHostFree(backup);
    } else {
      (void)hipFree(backup);
    }
  };
  auto restore = [&]() -> int {
    hipError_t e = copy_all(false);
    if (e != hipSuccess) return hip_fail(s, e, "autotune restore");
    s->cur = cur0;
    s->step = step0;
    s->keys_valid = false;
    s->have_binning = false;
    HIPCHK(s, launch_set_ctrl(s->dev, s->L, step0, cur0, s->R, 1));
    return MPC_OK;
  };
  hipError_t e0 = copy_all(true);
  if (e0 != hipSuccess) {
    release();
    return hip_fail(s, e0, "autotune backup");
  }
  // one trial: set the tiling, one untimed step (binning prologue), then
  // trial_steps timed steps; returns the fastest step in milliseconds (the
  // minimum is robust to a step slowed by other work on the device)
  std::vector<hipEvent_t> ev((size_t)trial_steps + 1, nullptr);
  auto trial = [&](int T, int g, int yb, int ord, double* ms) -> int {
    int r = mpc_set_tiling(s, T, g, yb, ord);
    if (r) return r;
    if ((r = restore())) return r;
    if ((r = ensure_keys(s))) return r;
    HIPCHK(s, enqueue_step(s, st));
    advance_mirror(s, 1);
    HIPCHK(s, hipEventRecord(ev[0], st));
    for (int32_t k = 0; k < trial_steps; ++k) {
      HIPCHK(s, enqueue_step(s, st));
      HIPCHK(s, hipEventRecord(ev[(size_t)k + 1], st));
    }
    HIPCHK(s, hipEventSynchronize(ev[(size_t)trial_steps]));
    advance_mirror(s, trial_steps);
    double m = 1e300;
    for (int32_t k = 0; k < trial_steps; ++k) {
      float f = 0.f;
      HIPCHK(s, hipEventElapsedTime(&f, ev[(size_t)k], ev[(size_t)k + 1]));
      m = std::min(m, (double)f);
    }
    *ms = m;
    return check_sticky(s);
  };
  rc = MPC_OK;
  for (hipEvent_t& x : ev)
    if (!rc && hipEventCreate(&x) != hipSuccess) rc = MPC_EHIP;
  int bestT = T0, bestG = g0, bestY = y0, bestO = o0;
  double best = 1e300;
  // coordinate search: tile size, then the persistent grid, then the row block
  const int Ts[] = {0, 8, 12, 16, 20, 22, 24, 28, 32};
  // grids: the resident maximum (0), fixed workgroups per CU (fewer waves
  // in flight per XCD can keep the gathered rows in L2), and oversubscribed
  // grids (freed slots take the remaining workgroups: better tail balance)
  const int full = s->num_cu * std::max(1, s->occupancy);
  const int gs[] = {0, 6 * s->num_cu, 8 * s->num_cu, 10 * s->num_cu, 2 * full, 16 * s->num_cu};
  const int ys[] = {8, 4, 16};
  for (int T : Ts) {
    double ms;
    if (rc || (rc = trial(T, 0, 8, 0, &ms))) break;
    if (ms < best) best = ms, bestT = T, bestG = 0, bestY = 8, bestO = 0;
  }
  for (int g : gs) {
    double ms;
    if (rc || g == 0) continue;
    if ((rc = trial(bestT, (g + 7) / 8 * 8, bestY, 0, &ms))) break;
    if (ms < best) best = ms, bestG = (g + 7) / 8 * 8;
  }
  for (int yb : ys) {
    double ms;
    if (rc || yb == 8) continue;
    if ((rc = trial(bestT, bestG, yb, 0, &ms))) break;
    if (ms < best) best = ms, bestY = yb;
  }
  // then the x-segment-major order with each row block
  for (int yb : ys) {
    double ms;
    if (rc) break;
    if ((rc = trial(bestT, bestG, yb, 1, &ms))) break;
    if (ms < best) best = ms, bestY = yb, bestO = 1;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  const std::string why = s->err;
  int rc2 = mpc_set_tiling(s, rc ? T0 : bestT, rc ? g0 : bestG, rc ? y0 : bestY, rc ? o0 : bestO);
  int rc3 = restore();
  release();
  if (rc) {
    s->err = "autotune: " + why;
    return rc;
  }
  if (rc2) return rc2;
  if (rc3) return rc3;
  if (tile_cells) *tile_cells = bestT;
  if (grid) *grid = (int32_t)s->L.collide_grid;
  return MPC_OK;
}

int mpc_run_noalloc(const mpc_params* p, double* x, double* v, int64_t n, uint64_t step,
                    int64_t nsteps, void* hip_stream) {
  if (!p || !x || !v || n < 1 || nsteps < 0) return MPC_EINVAL;
  if (p->form != MPC_FP64) return MPC_EINVAL;
  Plan P;
  std::string why;
  int rc = make_plan(p, 1, P, &why);
  if (rc) return rc;
  if ((uint64_t)n != P.box[0].n) return MPC_EINVAL;
  if (P.total > kScratchBytes) return MPC_ERANGE;
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  mpc_sim* s = nullptr;
  if ((rc = mpc_create(p, 1, ws, kScratchBytes, hip_stream, &s))) return rc;
  auto done = [&](int code) {
    (void)mpc_destroy(s);
    return code;
  };
  s->use_graph = false;  // kernel by kernel: graph instantiation may allocate
  const double a = p->a;
  if (launch_load_f64(s->dev, s->L, x, v, (uint32_t)n, a, 0) != hipSuccess)
    return done(MPC_EHIP);
  if ((rc = check_sticky(s))) return done(rc == MPC_ESTATE ? MPC_EINVAL : rc);
  if ((rc = mpc_set_step(s, step))) return done(rc);
  if ((rc = mpc_step(s, nsteps))) return done(rc);
  if ((rc = check_sticky(s))) return done(rc);
  if (launch_store_f64(s->dev, s->L, x, v, (uint32_t)n, a, s->cur) != hipSuccess ||
      hipStreamSynchronize(s->L.stream) != hipSuccess)
    return done(MPC_EHIP);
  return done(MPC_OK);
}

}  // extern "C"
