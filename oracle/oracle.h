/*
 * oracle.h -- plain single-threaded FP64 CPU oracle of one MPC-SRD time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * path.  Every function follows the paper's statement of the method
 * (Westphal, Goh, Winkler, Gompper, "HTMPC", arXiv:2406.15236):
 *   Sec. II Eq.(1)  ballistic streaming            -> orc_stream
 *   Sec. II         random shift of the cell grid  -> orc_shift
 *   Sec. II         sorting particles into cells   -> orc_keys, orc_sort
 *   Sec. II Eq.(2)  SRD rotation about random axis -> orc_collide
 *   Sec. II Eqs.(3)-(4) angular-momentum conserving SRD+a -> orc_collide
 *   Sec. II (Thermostat) MBS scaling, Gamma law    -> orc_collide / orc_gamma
 *   Sec. II (Boundary conditions) bounce-back, phantom particles, moving and
 *                   slip walls, Lees-Edwards shear of a periodic box
 *   Sec. II (External fields) constant gravity
 *   Sec. III.B.3 (Permanent exchange) reorder by cell -> orc_reorder
 *   Sec. III.C      fixed-point cell sums (optional)  -> orc_collide
 * Where the paper is silent, each function below states the reading it takes.
 *
 * Units: lengths in units of the cell size a (so a = 1 here); the caller
 * converts.  Arrays are SoA: x[0..n) is the x component, x[n..2n) y,
 * x[2n..3n) z; the same for v.
 */
#ifndef MPC_ORACLE_H
#define MPC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t  L[3];      /* box in cells; with walls L[2] = H, the fluid height   */
  int32_t  walls;     /* 1: no-slip walls at z = 0 and z = H (bounce-back)     */
  int32_t  mbs;       /* 1: Maxwell-Boltzmann-scaling thermostat              */
  int32_t  amc;       /* 1: cell angular momentum conserved (SRD+a, Eqs. 3-4);
                         periodic boxes or slip walls (no phantoms); with mbs
                         the scaling follows the correction                   */
  int32_t  fixed;     /* 1: cell sums of fluid terms in fixed point (Sec.
                         III.C, reproducibility): independent of the order  */
  int32_t  slip;      /* with walls, 1: slip walls (specular reflection, no
                         phantom particles) instead of no-slip walls         */
  double   h;         /* MPC time step                                         */
  double   alpha;     /* rotation angle, radians                               */
  double   kT;        /* k_B T                                                 */
  double   mass;      /* particle mass m                                       */
  double   density;   /* <N_c>, mean particles per cell (phantom fill)         */
  double   g[3];      /* constant acceleration (gravity), applied as a kick    */
  uint64_t seed;      /* Philox key                                            */
  double   uwall;     /* no-slip walls: the wall at z = H moves with velocity
                         +uwall along x, the wall at z = 0 with -uwall      */
  double   le_u;      /* periodic box, Lees-Edwards shear: the image above
                         (z + L_z) moves with +le_u along x; 0 = plain      */
} orc_params;

/* Per-cell diagnostics written by orc_collide when cell_out != NULL
 * (ORC_CELL_STRIDE doubles per cell, indexed by cell key). */
enum {
  ORC_C_NFLUID = 0, ORC_C_NPHANTOM, ORC_C_VX, ORC_C_VY, ORC_C_VZ, ORC_C_K,
  ORC_C_NX, ORC_C_NY, ORC_C_NZ, ORC_C_KAPPA, ORC_C_EK, ORC_C_ATTEMPTS,
  ORC_C_PX, ORC_C_PY, ORC_C_PZ, ORC_C_KPOST,
  ORC_CELL_STRIDE
};

/* Random-stream tags (counter word 3). */
enum { ORC_TAG_SHIFT = 1, ORC_TAG_AXIS = 2, ORC_TAG_THERMO = 3, ORC_TAG_PHANTOM = 4 };

/* Philox4x32-10 block function. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform conversions of Philox words: u24 = (w >> 8) 2^-24 in [0, 1);
 * u53 = (a:b top 53 bits) 2^-53 in [0, 1); u53_open = (m + 1/2) 2^-52 with
 * m the top 52 bits, in (0, 1); u32_open = (w + 1/2) 2^-32 in (0, 1). */
double orc_u24(uint32_t w);
double orc_u53(uint32_t a, uint32_t b);
double orc_u53_open(uint32_t a, uint32_t b);
double orc_u32_open(uint32_t w);

/* Grid shift of step t, s_k in [-1/2, 1/2) on a 2^-24 grid. */
void orc_shift(const orc_params* p, uint64_t t, double s[3]);

/* Number of collision cells (walls add the two wall-cut layers). */
int64_t orc_ncells(const orc_params* p);

/* Eq.(1) + boundary conditions, in place.  Returns the number of bounces. */
int64_t orc_stream(const orc_params* p, uint64_t t, int64_t n, double* x, double* v);

/* Cell key of every particle after the shift of step t.  Returns 0, or -1 if
 * a position is not finite / outside the box (key set to 0). */
int orc_keys(const orc_params* p, uint64_t t, int64_t n, const double* x, uint32_t* key);

/* Stable counting sort: offset[ncell+1] exclusive prefix of the counts,
 * perm[j] = storage index of the j-th particle in (key, index) order. */
void orc_sort(int64_t n, const uint32_t* key, int64_t ncell, uint32_t* perm, uint32_t* offset);

/* Wall volume fraction of a shifted z layer index cz in [-1, H] (0 if none). */
double orc_wall_fraction(const orc_params* p, double sz, int32_t cz);

/* Random axis of a cell (uniform on the unit sphere). */
void orc_cell_axis(const orc_params* p, uint64_t t, uint32_t key, double n[3]);

/* Gamma(shape, 1) variate of a cell by Marsaglia-Tsang; *attempts receives the
 * number of attempts used (0 means the attempt cap was hit: value 0). */
double orc_cell_gamma(const orc_params* p, uint64_t t, uint32_t key, double shape, int32_t* attempts);

/* Phantom particles of a wall-cut cell: returns the count (<= max_out) and
 * writes their velocities to vout[3*q + k]. */
int32_t orc_phantoms(const orc_params* p, uint64_t t, uint32_t key, double fw,
                     double* vout, int32_t max_out);

/* Rotation of u by angle alpha about unit axis n (right-handed). */
void orc_rotate(double alpha, const double n[3], const double u[3], double out[3]);

/* Collision of step t on already streamed velocities v, given the sort.
 * x (post-stream positions) is read only with p->amc (it may be NULL
 * otherwise); cell_out (optional) receives ORC_CELL_STRIDE doubles per cell.
 * Lees-Edwards (p->le_u) also reads x.  Returns -2 for amc with no-slip walls or
 * without x, for le_u with walls or without x, -3 (p->fixed) for a summand
 * outside the fixed-point range |x| < 2^37. */
int orc_collide(const orc_params* p, uint64_t t, int64_t n, const double* x, double* v,
                const uint32_t* perm, const uint32_t* offset, int64_t ncell,
                double* cell_out);

/* x, v <- x[perm], v[perm]. */
void orc_reorder(int64_t n, double* x, double* v, const uint32_t* perm);

/* One full step t -> t+1 on (x, v).  If reorder != 0 the arrays are permuted
 * into cell order afterwards.  key/perm/offset (optional) receive the binning
 * of this step (key indexed by the pre-step storage order). */
int orc_step(const orc_params* p, uint64_t t, int64_t n, double* x, double* v,
             int32_t reorder, uint32_t* key, uint32_t* perm, uint32_t* offset);

/* Observables: out[0..2] total momentum, out[3] kinetic energy,
 * out[4] temperature from the peculiar velocities, out[5] N. */
void orc_observables(const orc_params* p, int64_t n, const double* v, double out[6]);

#ifdef __cplusplus
}
#endif
#endif
