// mpc_internal.h -- layouts shared by the host planner and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

constexpr int kThreads = 256;               // threads per workgroup (4 wave64)
constexpr int kCollideThreads = 64;         // collide workgroup: one wave64
constexpr int kTileCap = 256;               // particles held in LDS per tile pass
constexpr int kTileMaxCells = 32;           // cells per collide tile (< kCollideThreads)
constexpr int kScanItems = 16;              // cells per thread in the scan kernels
constexpr int kScanBlock = kThreads * kScanItems;
constexpr int kPartBlock = kThreads * 4;    // particles per block of per-particle kernels

// Random-stream tags (counter word 3); counter = {draw, id, step, tag}.
enum : uint32_t { kTagShift = 1, kTagAxis = 2, kTagThermo = 3, kTagPhantom = 4,
                  kTagInitPos = 5, kTagInitVel = 6 };

// Sticky error bits in Ctrl::err.
enum : uint32_t { kErrKey = 1u, kErrCellOverflow = 2u, kErrFixRange = 4u };

enum : int { kFormF64 = 0, kFormF32 = 1, kFormSplit = 2 };

// Split form packs the unshifted cell as x | y << 11 | z << 22.
constexpr uint32_t kSplitXBits = 11, kSplitYBits = 11, kSplitZBits = 10;

struct BoxDev {
  int32_t L[3];        // cells per axis (walls: L[2] = H)
  int32_t nlz;         // z layers in key space: L[2], or H + 2 with walls
  uint32_t pbase, np;  // particle range in the flattened index space
  uint32_t cbase, nc;  // cell range in the flattened key space
  uint32_t key_lo, key_hi;
  uint32_t walls, mbs;
  double Ld[3];        // L as double
  float Lf[3];         // L as float
  double h;            // time step
  float hf;
  float pad0;
  double ca, sa, omc;  // cos(alpha), sin(alpha), 1 - cos(alpha)
  double kT, mass, density, sd;  // sd = sqrt(kT / m)
  double gh[3];        // g * h
  uint32_t grav;
  uint32_t wcbase;     // walls: first index of this box's cells of the two
                       // wall-cut layers (2 L0 L1 per box) in a flat index space
  uint32_t slip;       // walls: specular reflection, no phantoms
  float uwf;           // uw as float
  double uw;           // no-slip walls: x velocity of the wall at z = H (cells per
                       // unit time); the wall at z = 0 moves with -uw
  uint32_t le;         // periodic z with Lees-Edwards shear
  float leuf;          // leu as float
  double leu;          // Lees-Edwards: x velocity of the image above the box
};

struct Tile {          // one collide work item: cells [c0, c0 + nc) of box `box`
  uint32_t c0;         // first global cell key
  uint16_t nc;
  uint16_t box;
  uint32_t x0, y0, z0; // coordinates of the first cell in its box (z0: key layer)
};

struct PBlock {        // one block of a per-particle kernel
  uint32_t box;
  uint32_t p0;         // first global particle index
};

struct Ctrl {          // device-resident step state, read by every kernel
  uint64_t step;       // step index t of the next step
  uint32_t cur;        // which state buffer holds the current state (flips every step)
  uint32_t err;        // sticky error bits
  int32_t reorder;     // R
  uint32_t pad[3];
};

struct CellDraw {       // random draws of one cell for the current step
  double n[3];         // rotation axis
  double Ek;           // thermostat target energy, 0 = no scaling
};

struct PhantomSums {   // phantom particles of an occupied wall-cut cell
  double v[3];         // sum of their velocities
  double v2;           // sum of |v|^2
  double n;            // their number
  double pad;
};

// Particle records, one per storage slot (array of structures): the collide
// gathers a particle with one or two 16-byte loads per 16 bytes of record, so
// that a run of consecutive slots is one contiguous span of memory instead of
// one span per component.  Positions and velocities are in cell units.
struct alignas(16) RecF64 {
  double x[3];
  double v[3];
};
struct alignas(8) RecF32 {
  float x[3];
  float v[3];
};
struct alignas(16) RecSplit {
  uint32_t cell;  // x | y << 11 | z << 22
  float o[3];     // offsets inside the cell, [0, 1)
  float v[3];
  uint32_t id;    // logical index of the particle in this slot
};
static_assert(sizeof(RecF64) == 48 && sizeof(RecF32) == 24 && sizeof(RecSplit) == 32,
              "record sizes");
constexpr size_t rec_bytes(int form) {
  return form == kFormF64 ? sizeof(RecF64) : (form == kFormF32 ? sizeof(RecF32) : sizeof(RecSplit));
}

// One state buffer.  Every step writes the state into the other buffer, cell
// by cell of the current step, and inside the particles of one tile pass
// grouped by their cell of the next step (so that the next step gathers
// contiguous runs).  The logical index of slot i (its index in the caller's
// order, renumbered to the (cell, index) order on reorder steps) is
// id[i * id_stride]: an array of its own for FP64 and FP32 (stride 1), the id
// word of the record for the split form (stride 8).
struct StatePtrs {
  void* rec;
  uint32_t* id;
  uint32_t id_stride;
};

struct Dev {           // device pointers carved from the workspace
  StatePtrs S[2];
  uint32_t* key;       // cell key per particle (storage order)
  uint16_t* rank;      // rank of the particle among those counted for its key
  uint32_t* perm;      // position in (cell, any order) -> stored slot
  uint32_t* hist;      // particles per cell of the next step; zeroed by the scan
  uint32_t* offset;    // exclusive prefix, ncell + 1
  uint32_t* scan_blk;  // per scan-block totals
  Ctrl* ctrl;
  BoxDev* boxes;
  Tile* tiles;
  PBlock* pblocks;
  double* partials;    // per-block observable partial sums
  CellDraw* draws;     // per-cell draws of the current step (written by the scan)
  PhantomSums* phs;    // walls only: phantom sums of wall-cut cells (written by the scan)
  uint32_t ntot;       // particles over all boxes (bound of every particle index)
};

struct Launch {
  int form;
  int round_phantoms;      // split form: phantom velocities rounded to FP32
  int walls, mbs, amc;     // feature flags (identical for all boxes)
  int fixed;               // fixed-point cell sums
  int le;                  // some box has Lees-Edwards shear
  uint32_t nbox;
  uint64_t ntot, ctot;     // particles, cells over all boxes
  uint32_t ntiles, npblocks, nscan;
  uint32_t collide_grid;
  uint32_t wcells;         // walls: cells of the wall-cut layers over all boxes
  int xcd_remap;
  hipStream_t stream;
};

// Launchers (mpc_kernels.hip).
hipError_t launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s);
hipError_t launch_key_hist(const Dev& d, const Launch& l);
hipError_t launch_scan(const Dev& d, const Launch& l);
hipError_t launch_scatter(const Dev& d, const Launch& l);
hipError_t launch_phantoms(const Dev& d, const Launch& l);
hipError_t launch_collide(const Dev& d, const Launch& l);
hipError_t launch_advance(const Dev& d, const Launch& l);
hipError_t launch_set_ctrl(const Dev& d, const Launch& l, uint64_t step, uint32_t cur,
                           int32_t reorder, int clear_err);
hipError_t launch_init_state(const Dev& d, const Launch& l, uint64_t seed);
hipError_t launch_obs_pass1(const Dev& d, const Launch& l);
hipError_t launch_obs_pass2(const Dev& d, const Launch& l, const double* vmean_dev);
hipError_t launch_remove_mean(const Dev& d, const Launch& l, const double* vmean_dev);
// inv: np entries filled with 0xffffffff by the caller (null: slots are the
// logical order); lidx: box-local logical indices; out: [6][m] FP64
hipError_t launch_gather_particles(const Dev& d, const Launch& l, const StatePtrs& S,
                                  uint32_t* inv, uint32_t pbase, uint32_t np,
                                  const uint32_t* lidx, uint32_t m, double* out);
// box 0, FP64 form: caller's device arrays (physical units) <-> state buffer cur
hipError_t launch_load_f64(const Dev& d, const Launch& l, const double* x, const double* v,
                           uint32_t n, double a, uint32_t cur);
hipError_t launch_store_f64(const Dev& d, const Launch& l, double* x, double* v, uint32_t n,
                            double a, uint32_t cur);
hipError_t launch_canon_perm(const Dev& d, const Launch& l, const StatePtrs& ids);
hipError_t collide_occupancy(const Launch& l, int* blocks_per_cu);  // flags of l only

}  // namespace mpc
