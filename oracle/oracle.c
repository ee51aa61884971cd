/*
 * oracle.c -- plain, slow, single-threaded FP64 CPU oracle of the MPC-SRD step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for readability against
 * the paper, not for speed: every loop runs over particles or cells in index
 * order, sums are sequential, nothing is blocked, fused or reordered beyond
 * what the method states.  Built with -O2 -ffp-contract=off so that each
 * written operation is one IEEE operation; fma() appears only where the
 * streaming rule below asks for it.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon, Moraes, Dror and Shaw,      */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two  */
/* 32x32->64 multiplications whose high halves are xored with the other two  */
/* counter words and the key; the key is advanced by the Weyl constants      */
/* before every round after the first.                                       */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t next[4];
    next[0] = (uint32_t)(prod1 >> 32) ^ c[1] ^ k[0];
    next[1] = (uint32_t)prod1;
    next[2] = (uint32_t)(prod0 >> 32) ^ c[3] ^ k[1];
    next[3] = (uint32_t)prod0;
    memcpy(c, next, sizeof c);
  }
  memcpy(out, c, sizeof c);
}

/* One draw of the method's random stream: counter {j, id, step, tag}, key = seed. */
static void draw(const orc_params* p, uint32_t j, uint32_t id, uint64_t t, uint32_t tag,
                 uint32_t w[4]) {
  uint32_t ctr[4] = {j, id, (uint32_t)t, tag};
  uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
  orc_philox(ctr, key, w);
}

double orc_u24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

double orc_u53(uint32_t a, uint32_t b) {
  uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
  return (double)m * 0x1p-53;
}

double orc_u53_open(uint32_t a, uint32_t b) {
  uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12); /* 52 bits */
  return (double)(2 * m + 1) * 0x1p-53;                    /* (m + 1/2) 2^-52 */
}

double orc_u32_open(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

static const double TWO_PI = 6.283185307179586;

/* ------------------------------------------------------------------------ */
/* Sec. II: the whole collision lattice is shifted at random before every     */
/* collision (Galilean invariance).  One shift vector per step, uniform in    */
/* [-a/2, a/2)^3 on a 2^-24 grid (reading: shift grid).                       */
/* ------------------------------------------------------------------------ */
void orc_shift(const orc_params* p, uint64_t t, double s[3]) {
  uint32_t w[4];
  draw(p, 0, 0, t, ORC_TAG_SHIFT, w);
  for (int k = 0; k < 3; ++k) s[k] = orc_u24(w[k]) - 0.5;
}

int64_t orc_ncells(const orc_params* p) {
  int64_t layers = p->walls ? (int64_t)p->L[2] + 2 : (int64_t)p->L[2];
  return (int64_t)p->L[0] * p->L[1] * layers;
}

/* Periodic wrap of one coordinate into [0, L) (reading: wrap corner). */
static double wrap(double x, double L) {
  if (x < 0.0) {
    x = x + L;
  } else if (x >= L) {
    x = x - L;
  }
  if (!(x >= 0.0 && x < L)) {
    if (x == L) {
      x = 0.0;
    } else if (isfinite(x)) {
      x = x - L * floor(x / L);
      if (x >= L || x < 0.0) x = 0.0;
    }
  }
  return x;
}

/* ------------------------------------------------------------------------ */
/* Sec. II Eq.(1): r <- r + h v.  No-slip walls (Sec. II, Boundary            */
/* conditions): a particle that crossed z = 0 or z = H is put back by         */
/* time-reversed bounce-back, r <- r_end - 2 v t_rem, v <- -v, where t_rem is */
/* the time spent beyond the wall (reading: bounce-back geometry).  A moving  */
/* wall (velocity u along x) reverses the velocity in its own frame:          */
/* v <- 2u - v, r <- r_end - 2 (v - u) t_rem.  Slip walls reflect            */
/* specularly: only v_z and z are mirrored.                                   */
/* ------------------------------------------------------------------------ */
/* Lees-Edwards shear (Sec. II, boundary conditions: periodic boundaries with
 * shear flow): at time tau the periodic image above the box (z + L_z) is
 * displaced by d(tau) = (U tau) mod L_x along x and moves with velocity U.
 * tau = t_end h, the end of the streaming of step t_end - 1. */
static double le_offset(const orc_params* p, uint64_t t_end) {
  double d = p->le_u * ((double)t_end * p->h);
  return d - (double)p->L[0] * floor(d / (double)p->L[0]);
}

/* Lees-Edwards frame of a particle in the collision of step t: +1 or -1 if
 * its shifted cell lies across the lower or upper z face (the cell is formed
 * with the image on the other side), else 0. */
static int le_side(const orc_params* p, double z, double sz) {
  double cz = floor(z + sz);
  return cz < 0.0 ? 1 : (cz >= (double)p->L[2] ? -1 : 0);
}

int64_t orc_stream(const orc_params* p, uint64_t t, int64_t n, double* x, double* v) {
  const double h = p->h;
  const double Lx = p->L[0], Ly = p->L[1], Lz = p->L[2];
  int64_t bounces = 0;
  for (int64_t i = 0; i < n; ++i) {
    double xe = fma(h, v[i], x[i]);
    double ye = fma(h, v[n + i], x[n + i]);
    double ze = fma(h, v[2 * n + i], x[2 * n + i]);
    if (p->walls) {
      int crossed = 0;
      double zw = 0.0;
      if (ze < 0.0) {
        crossed = 1;
        zw = 0.0;
      } else if (ze > Lz) {
        crossed = 1;
        zw = Lz;
      }
      if (crossed) {
        double vz = v[2 * n + i];
        double tr2 = 2.0 * ((ze - zw) / vz);
        if (p->slip) {
          ze = ze - tr2 * vz;
        } else {
          double uw = zw == 0.0 ? -p->uwall : p->uwall;
          xe = xe - tr2 * (v[i] - uw);
          ye = ye - tr2 * v[n + i];
          ze = ze - tr2 * vz;
          v[i] = 2.0 * uw - v[i];
          v[n + i] = -v[n + i];
        }
        if (ze < 0.0) ze = 0.0;
        if (ze > Lz) ze = Lz;
        v[2 * n + i] = -v[2 * n + i];
        ++bounces;
      }
    } else {
      if (p->le_u != 0.0 && (ze >= Lz || ze < 0.0)) {
        /* through the sheared face: into the frame of the image it came from */
        double d = le_offset(p, t + 1);
        if (ze >= Lz) {
          xe = xe - d;
          v[i] = v[i] - p->le_u;
        } else {
          xe = xe + d;
          v[i] = v[i] + p->le_u;
        }
      }
      ze = wrap(ze, Lz);
    }
    x[i] = wrap(xe, Lx);
    x[n + i] = wrap(ye, Ly);
    x[2 * n + i] = ze;
  }
  return bounces;
}

/* ------------------------------------------------------------------------ */
/* Sec. II: sort particles into the cubic cells of the shifted lattice.       */
/* Cell c_k = floor(x_k + s_k) (exact: s is on a 2^-24 grid), periodic axes   */
/* wrap c into [0, L); with walls the z layer c_z + 1 lies in [0, H+1].       */
/* key = (c_z * L_y + c_y) * L_x + c_x (reading: x-fastest linear key).       */
/* ------------------------------------------------------------------------ */
int orc_keys(const orc_params* p, uint64_t t, int64_t n, const double* x, uint32_t* key) {
  double s[3];
  orc_shift(p, t, s);
  int rc = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t c[3];
    int ok = 1;
    for (int k = 0; k < 3; ++k) {
      double y = x[k * n + i] + s[k];
      if (!(y >= -2.0 && y < (double)p->L[k] + 2.0)) {
        ok = 0;
        c[k] = 0;
        continue;
      }
      c[k] = (int64_t)floor(y);
    }
    if (ok && !p->walls && p->le_u != 0.0 && (c[2] < 0 || c[2] >= p->L[2])) {
      /* Lees-Edwards: a cell across a z face is formed with the image on the
       * other side, displaced by -/+ d along x */
      double d = le_offset(p, t + 1);
      double xi = c[2] >= p->L[2] ? x[i] - d : x[i] + d;
      int64_t cx = (int64_t)floor(xi + s[0]) % p->L[0];
      c[0] = cx < 0 ? cx + p->L[0] : cx;
    }
    if (ok) {
      for (int k = 0; k < 2; ++k) {
        if (c[k] < 0) c[k] += p->L[k];
        else if (c[k] >= p->L[k]) c[k] -= p->L[k];
      }
      if (p->walls) {
        c[2] += 1;
        if (c[2] < 0 || c[2] > (int64_t)p->L[2] + 1) ok = 0;
      } else {
        if (c[2] < 0) c[2] += p->L[2];
        else if (c[2] >= p->L[2]) c[2] -= p->L[2];
      }
      for (int k = 0; k < 2; ++k)
        if (c[k] < 0 || c[k] >= p->L[k]) ok = 0;
      if (!p->walls && (c[2] < 0 || c[2] >= p->L[2])) ok = 0;
    }
    if (!ok) {
      rc = -1;
      key[i] = 0;
      continue;
    }
    key[i] = (uint32_t)((c[2] * p->L[1] + c[1]) * p->L[0] + c[0]);
  }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Counting sort (the pattern of Sec. III.B.2-3: count per cell, prefix sum   */
/* as cell offsets, then place each particle).  Particles are visited in      */
/* ascending storage index, so equal keys keep their storage order.           */
/* ------------------------------------------------------------------------ */
void orc_sort(int64_t n, const uint32_t* key, int64_t ncell, uint32_t* perm, uint32_t* offset) {
  uint32_t* count = (uint32_t*)calloc((size_t)ncell + 1, sizeof(uint32_t));
  for (int64_t i = 0; i < n; ++i) count[key[i]] += 1;
  uint32_t run = 0;
  for (int64_t c = 0; c < ncell; ++c) {
    offset[c] = run;
    run += count[c];
  }
  offset[ncell] = run;
  memset(count, 0, ((size_t)ncell + 1) * sizeof(uint32_t));
  for (int64_t i = 0; i < n; ++i) {
    uint32_t c = key[i];
    perm[offset[c] + count[c]] = (uint32_t)i;
    count[c] += 1;
  }
  free(count);
}

/* ------------------------------------------------------------------------ */
/* Wall-cut layers (Sec. II, Boundary conditions): with shift s_z the layer   */
/* c_z spans [c_z - s_z, c_z + 1 - s_z).  For s_z >= 0 layer 0 reaches s_z    */
/* into the bottom wall and layer H lies 1 - s_z inside the top wall; for     */
/* s_z < 0 those are layers -1 (1 + s_z in the wall) and H-1 (-s_z).          */
/* ------------------------------------------------------------------------ */
double orc_wall_fraction(const orc_params* p, double sz, int32_t cz) {
  if (!p->walls) return 0.0;
  int32_t H = p->L[2];
  if (sz >= 0.0) {
    if (cz == 0) return sz;
    if (cz == H) return 1.0 - sz;
  } else {
    if (cz == -1) return 1.0 + sz;
    if (cz == H - 1) return -sz;
  }
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Sec. II: rotation axis chosen at random, independently for every cell and  */
/* step: z uniform in (-1, 1], azimuth uniform in [0, 2 pi) gives a uniform   */
/* direction on the sphere (reading: axis law).                               */
/* ------------------------------------------------------------------------ */
void orc_cell_axis(const orc_params* p, uint64_t t, uint32_t key, double n[3]) {
  uint32_t w[4];
  draw(p, 0, key, t, ORC_TAG_AXIS, w);
  double u1 = orc_u53(w[0], w[1]);
  double u2 = orc_u53(w[2], w[3]);
  double z = 1.0 - 2.0 * u1;
  double r = sqrt(1.0 - z * z);
  double phi = TWO_PI * u2;
  n[0] = r * cos(phi);
  n[1] = r * sin(phi);
  n[2] = z;
}

/* ------------------------------------------------------------------------ */
/* Sec. II (Thermostat): E_k follows a Gamma law of shape f/2 and scale kT.   */
/* Gamma(shape, 1) by Marsaglia and Tsang (ACM TOMS 26, 2000): with           */
/* d = shape - 1/3, c = 1/sqrt(9d), draw a normal z and a uniform u, set      */
/* v = (1 + c z)^3, accept d v if v > 0 and                                   */
/* log u < z^2/2 + d - d v + d log v.  Attempt j uses draw j of the cell's    */
/* THERMO stream: Box-Muller (cosine branch) from words 0,1 and the uniform   */
/* from words 2,3.  At most 64 attempts (reading: gamma attempt cap).         */
/* ------------------------------------------------------------------------ */
double orc_cell_gamma(const orc_params* p, uint64_t t, uint32_t key, double shape,
                      int32_t* attempts) {
  double d = shape - 1.0 / 3.0;
  double c = 1.0 / sqrt(9.0 * d);
  for (uint32_t j = 0; j < 64; ++j) {
    uint32_t w[4];
    draw(p, j, key, t, ORC_TAG_THERMO, w);
    double u1 = orc_u32_open(w[0]);
    double u2 = (double)w[1] * 0x1p-32;
    double z = sqrt(-2.0 * log(u1)) * cos(TWO_PI * u2);
    double vv = 1.0 + c * z;
    if (vv <= 0.0) continue;
    vv = vv * vv * vv;
    double u = orc_u53_open(w[2], w[3]);
    double lhs = log(u);
    double rhs = 0.5 * z * z + d - d * vv + d * log(vv);
    if (lhs < rhs) {
      *attempts = (int32_t)j + 1;
      return d * vv;
    }
  }
  *attempts = 0;
  return 0.0;
}

/* Normal number m of a cell's PHANTOM stream: draw 1 + m/4, Box-Muller pair
 * (m%4)/2 (words 2p, 2p+1), cosine branch for even m, sine branch for odd. */
static double phantom_normal(const orc_params* p, uint64_t t, uint32_t key, uint32_t m) {
  uint32_t w[4];
  draw(p, 1 + m / 4, key, t, ORC_TAG_PHANTOM, w);
  uint32_t pair = (m % 4) / 2;
  double r = sqrt(-2.0 * log(orc_u32_open(w[2 * pair])));
  double th = TWO_PI * ((double)w[2 * pair + 1] * 0x1p-32);
  return (m % 2 == 0) ? r * cos(th) : r * sin(th);
}

/* ------------------------------------------------------------------------ */
/* Sec. II (Boundary conditions): the wall part of a cut cell is filled with  */
/* phantom particles so that the whole cell holds <N_c> on average; their     */
/* velocities are Gaussian, zero mean, variance kT/m (reading: phantom        */
/* spread).  Count ~ Poisson(<N_c> f_w) by inversion on draw 0 (reading:      */
/* phantom count), truncated at 127.                                          */
/* ------------------------------------------------------------------------ */
int32_t orc_phantoms(const orc_params* p, uint64_t t, uint32_t key, double fw, double* vout,
                     int32_t max_out) {
  double lam = p->density * fw;
  uint32_t w[4];
  draw(p, 0, key, t, ORC_TAG_PHANTOM, w);
  double u = orc_u53(w[0], w[1]);
  int32_t k = 0;
  double pk = exp(-lam);
  double F = pk;
  while (u >= F && k < 127) {
    k += 1;
    pk = pk * lam / (double)k;
    F = F + pk;
  }
  if (k > max_out) k = max_out;
  double sd = sqrt(p->kT / p->mass);
  for (int32_t q = 0; q < k; ++q)
    for (int32_t a = 0; a < 3; ++a)
      vout[3 * q + a] = sd * phantom_normal(p, t, key, (uint32_t)(3 * q + a));
  return k;
}

/* Rodrigues' formula, right-handed rotation by alpha about the unit vector n:
 * u' = cos(a) u + sin(a) (n x u) + (1 - cos(a)) (n . u) n. */
static void rotate_cs(double ca, double sa, double omc, const double n[3], const double u[3],
                      double out[3]) {
  double ndu = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
  double cr[3] = {n[1] * u[2] - n[2] * u[1], n[2] * u[0] - n[0] * u[2],
                  n[0] * u[1] - n[1] * u[0]};
  double f = omc * ndu;
  for (int k = 0; k < 3; ++k) out[k] = ca * u[k] + sa * cr[k] + f * n[k];
}

void orc_rotate(double alpha, const double n[3], const double u[3], double out[3]) {
  double ca = cos(alpha);
  rotate_cs(ca, sin(alpha), 1.0 - ca, n, u, out);
}

/* ------------------------------------------------------------------------ */
/* Sec. II Eq.(2) with the MBS thermostat: per cell, v_cm = sum m v / M over  */
/* the cell (phantoms included), relative velocities rotated by alpha about   */
/* the cell's axis and scaled by kappa = sqrt(2 E_k / sum m v_c^2).           */
/* Cells with fewer than two particles are left unchanged.  Afterwards the    */
/* gravity kick v <- v + g h is applied to every particle (reading: gravity). */
/* ------------------------------------------------------------------------ */
/* One cell sum (Sec. III.C, reproducibility).  Without p->fixed: FP64
 * additions in the order the terms come.  With p->fixed: each term x is the
 * integer trunc(x 2^80) (a 128-bit integer with 80 fractional bits), the sum
 * is the exact integer sum, and its value is that integer rounded once to the
 * nearest double, times 2^-80; it does not depend on the order of the terms.
 * Terms need |x| < 2^37, so that no sum of at most 2^10 terms can overflow;
 * a larger term sets *bad. */
typedef struct {
  int fixed;
  double d;
  __int128 s;
} orc_sum;

static orc_sum sum_new(const orc_params* p) {
  orc_sum a;
  a.fixed = p->fixed;
  a.d = 0.0;
  a.s = 0;
  return a;
}

static void sum_add(orc_sum* a, double x, int* bad) {
  if (!a->fixed) {
    a->d = a->d + x;
  } else if (fabs(x) < 0x1p37) {
    a->s += (__int128)(x * 0x1p80);
  } else {
    *bad = 1;
  }
}

static double sum_val(const orc_sum* a) { return a->fixed ? (double)a->s * 0x1p-80 : a->d; }

/* Sec. II Eqs.(3)-(4), SRD+a: after the rotation, each particle also gets
 * omega x r_ic, with r_ic its position relative to the cell's centre of mass
 * and omega = m I^-1 sum_i r_ic x (u_i - D u_i) (u_i = v_i - v_cm, D the
 * rotation, I the cell's inertia tensor about the centre of mass), so that
 * the cell's angular momentum about its centre of mass is unchanged.
 * Positions are taken in the cell's frame, (x + s) - floor(x + s), which has
 * no periodic-image ambiguity.  Readings: a cell of two particles has a
 * singular I; the change of angular momentum then lies in I's range and the
 * pseudo-inverse, omega = dL / (m |r_1 - r_2|^2 / 2), is used; three or more
 * particles use I^-1 (Cramer's rule), and omega = 0 if det I = 0.  Periodic
 * boxes or slip walls only (phantom particles carry no positions).  With the thermostat, the
 * scaling is applied to the corrected relative velocities (see orc_collide). */
static void amc_cell(const orc_params* p, const double s[3], int64_t n, const double* x,
                     const double* v0, double* v, const uint32_t* perm, uint32_t b, uint32_t e,
                     const double V[3], const double ax[3], double ca, double sa, double omc,
                     int* bad) {
  const double m = p->mass;
  const int64_t nf = (int64_t)e - (int64_t)b;
  orc_sum rs[3] = {sum_new(p), sum_new(p), sum_new(p)};
  for (uint32_t j = b; j < e; ++j) {
    uint32_t i = perm[j];
    for (int k = 0; k < 3; ++k) {
      double y = x[k * n + i] + s[k];
      sum_add(&rs[k], y - floor(y), bad);
    }
  }
  double rc[3];
  for (int k = 0; k < 3; ++k) rc[k] = sum_val(&rs[k]) / (double)nf;
  orc_sum dLs[3], Is[9];
  for (int k = 0; k < 3; ++k) dLs[k] = sum_new(p);
  for (int k = 0; k < 9; ++k) Is[k] = sum_new(p);
  for (uint32_t j = b; j < e; ++j) {
    uint32_t i = perm[j];
    double r[3], u[3], d[3], w[3];
    for (int k = 0; k < 3; ++k) {
      double y = x[k * n + i] + s[k];
      r[k] = (y - floor(y)) - rc[k];
      u[k] = v0[k * n + i] - V[k];
    }
    rotate_cs(ca, sa, omc, ax, u, d);
    for (int k = 0; k < 3; ++k) w[k] = u[k] - d[k];
    sum_add(&dLs[0], m * (r[1] * w[2] - r[2] * w[1]), bad);
    sum_add(&dLs[1], m * (r[2] * w[0] - r[0] * w[2]), bad);
    sum_add(&dLs[2], m * (r[0] * w[1] - r[1] * w[0]), bad);
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) sum_add(&Is[3 * a + c], m * ((a == c ? r2 : 0.0) - r[a] * r[c]), bad);
  }
  double dL[3], I[9];
  for (int k = 0; k < 3; ++k) dL[k] = sum_val(&dLs[k]);
  for (int k = 0; k < 9; ++k) I[k] = sum_val(&Is[k]);
  double om[3] = {0.0, 0.0, 0.0};
  if (nf == 2) {
    uint32_t i1 = perm[b], i2 = perm[b + 1];
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double y1 = x[k * n + i1] + s[k], y2 = x[k * n + i2] + s[k];
      double dd = (y1 - floor(y1)) - (y2 - floor(y2));
      d2 = d2 + dd * dd;
    }
    if (d2 > 0.0)
      for (int k = 0; k < 3; ++k) om[k] = dL[k] / (m * d2 / 2.0);
  } else {
    double det = I[0] * (I[4] * I[8] - I[5] * I[7]) - I[1] * (I[3] * I[8] - I[5] * I[6]) +
                 I[2] * (I[3] * I[7] - I[4] * I[6]);
    if (det != 0.0) {
      for (int k = 0; k < 3; ++k) {
        double A[9];
        memcpy(A, I, sizeof A);
        for (int a = 0; a < 3; ++a) A[3 * a + k] = dL[a];
        double dk = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                    A[2] * (A[3] * A[7] - A[4] * A[6]);
        om[k] = dk / det;
      }
    }
  }
  for (uint32_t j = b; j < e; ++j) {
    uint32_t i = perm[j];
    double r[3];
    for (int k = 0; k < 3; ++k) {
      double y = x[k * n + i] + s[k];
      r[k] = (y - floor(y)) - rc[k];
    }
    double oxr[3] = {om[1] * r[2] - om[2] * r[1], om[2] * r[0] - om[0] * r[2],
                     om[0] * r[1] - om[1] * r[0]};
    for (int k = 0; k < 3; ++k) v[k * n + i] = v[k * n + i] + oxr[k];
  }
}

int orc_collide(const orc_params* p, uint64_t t, int64_t n, const double* x, double* v,
                const uint32_t* perm, const uint32_t* offset, int64_t ncell, double* cell_out) {
  if (p->amc && ((p->walls && !p->slip) || !x)) return -2;
  if (p->le_u != 0.0 && (p->walls || !x)) return -2;
  int bad = 0; /* a fixed-point summand out of range */
  const double m = p->mass;
  double* v0 = NULL; /* pre-collision velocities (SRD+a) */
  if (p->amc) {
    v0 = (double*)malloc((size_t)3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    memcpy(v0, v, (size_t)3 * (size_t)n * sizeof(double));
  }
  const double ca = cos(p->alpha), sa = sin(p->alpha), omc = 1.0 - ca;
  double s[3];
  orc_shift(p, t, s);
  /* SRD+a with Lees-Edwards shear: the positions of the particles that a cell
   * across a z face takes as their image, x -/+ d (the velocities get their
   * frame change in the cell loop) */
  double* xa = (double*)x;
  if (p->amc && p->le_u != 0.0) {
    xa = (double*)malloc((size_t)3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    memcpy(xa, x, (size_t)3 * (size_t)n * sizeof(double));
    double d = le_offset(p, t + 1);
    for (int64_t i = 0; i < n; ++i) {
      int side = le_side(p, x[2 * n + i], s[2]);
      if (side < 0) xa[i] = x[i] - d;
      if (side > 0) xa[i] = x[i] + d;
    }
  }
  const int64_t plane = (int64_t)p->L[0] * p->L[1];
  enum { PMAX = 127 };
  double vp[3 * PMAX];
  if (cell_out) memset(cell_out, 0, (size_t)ncell * ORC_CELL_STRIDE * sizeof(double));

  for (int64_t c = 0; c < ncell; ++c) {
    uint32_t b = offset[c], e = offset[c + 1];
    int64_t nf = (int64_t)e - (int64_t)b;
    if (nf == 0) continue;

    int32_t np = 0;
    if (p->walls && !p->slip) {
      int32_t cz = (int32_t)(c / plane) - 1;
      double fw = orc_wall_fraction(p, s[2], cz);
      if (fw > 0.0) {
        np = orc_phantoms(p, t, (uint32_t)c, fw, vp, PMAX);
        /* phantoms move with the wall whose part of the cell they fill: the
         * layer cut by z = 0 is c_z = 0 (s_z >= 0) or c_z = -1 (s_z < 0) */
        int32_t bottom = cz == (s[2] >= 0.0 ? 0 : -1);
        double uw = bottom ? -p->uwall : p->uwall;
        for (int32_t q = 0; q < np; ++q) vp[3 * q] = vp[3 * q] + uw;
      }
    }
    int64_t ntot = nf + np;
    /* Lees-Edwards: the particles of a colliding cell across a z face take the
     * velocity frame of the image they are mapped to (v_x - U above the upper
     * face, + U below the lower one) for the collision, and leave it after */
    const int le = p->le_u != 0.0 && ntot >= 2;
    if (le) {
      for (uint32_t j = b; j < e; ++j) {
        uint32_t i = perm[j];
        int side = le_side(p, x[2 * n + i], s[2]);
        if (side < 0) v[i] = v[i] - p->le_u;
        if (side > 0) v[i] = v[i] + p->le_u;
        if (v0 && side < 0) v0[i] = v0[i] - p->le_u;
        if (v0 && side > 0) v0[i] = v0[i] + p->le_u;
      }
    }

    orc_sum Ps[3] = {sum_new(p), sum_new(p), sum_new(p)};
    for (uint32_t j = b; j < e; ++j) {
      uint32_t i = perm[j];
      for (int k = 0; k < 3; ++k) sum_add(&Ps[k], m * v[k * n + i], &bad);
    }
    /* phantoms follow in their draw order */
    double P[3] = {sum_val(&Ps[0]), sum_val(&Ps[1]), sum_val(&Ps[2])};
    for (int32_t q = 0; q < np; ++q)
      for (int k = 0; k < 3; ++k) P[k] = P[k] + m * vp[3 * q + k];
    double M = (double)ntot * m;
    double V[3] = {P[0] / M, P[1] / M, P[2] / M};

    orc_sum Ks = sum_new(p);
    for (uint32_t j = b; j < e; ++j) {
      uint32_t i = perm[j];
      double dx = v[i] - V[0], dy = v[n + i] - V[1], dz = v[2 * n + i] - V[2];
      sum_add(&Ks, m * (dx * dx + dy * dy + dz * dz), &bad);
    }
    double K = sum_val(&Ks);
    for (int32_t q = 0; q < np; ++q) {
      double dx = vp[3 * q] - V[0], dy = vp[3 * q + 1] - V[1], dz = vp[3 * q + 2] - V[2];
      K = K + m * (dx * dx + dy * dy + dz * dz);
    }

    double* co = cell_out ? cell_out + c * ORC_CELL_STRIDE : NULL;
    if (co) {
      co[ORC_C_NFLUID] = (double)nf;
      co[ORC_C_NPHANTOM] = (double)np;
      co[ORC_C_VX] = V[0];
      co[ORC_C_VY] = V[1];
      co[ORC_C_VZ] = V[2];
      co[ORC_C_K] = K;
      co[ORC_C_KAPPA] = 1.0;
      co[ORC_C_PX] = P[0];
      co[ORC_C_PY] = P[1];
      co[ORC_C_PZ] = P[2];
    }
    if (ntot < 2) continue;

    double ax[3];
    orc_cell_axis(p, t, (uint32_t)c, ax);
    double kappa = 1.0, Ek = 0.0;
    int have_ek = 0;
    if (p->mbs && K > 0.0) {
      int32_t att = 0;
      double gv = orc_cell_gamma(p, t, (uint32_t)c, 1.5 * (double)(ntot - 1), &att);
      if (att > 0) {
        Ek = p->kT * gv;
        have_ek = 1;
        kappa = sqrt((2.0 * Ek) / K);
        if (co) co[ORC_C_EK] = Ek;
      }
      if (co) co[ORC_C_ATTEMPTS] = (double)att;
    }

    /* SRD+a: the rotation is unscaled; the thermostat scales the relative
     * velocities after the angular-momentum correction (below) */
    const double kr = p->amc ? 1.0 : kappa;
    double Kpost = 0.0;
    for (uint32_t j = b; j < e; ++j) {
      uint32_t i = perm[j];
      double u[3] = {v[i] - V[0], v[n + i] - V[1], v[2 * n + i] - V[2]};
      double up[3];
      rotate_cs(ca, sa, omc, ax, u, up);
      for (int k = 0; k < 3; ++k) {
        v[k * n + i] = V[k] + kr * up[k];
        Kpost = Kpost + m * (kr * up[k]) * (kr * up[k]);
      }
    }
    if (p->amc) {
      amc_cell(p, s, n, xa, v0, v, perm, b, e, V, ax, ca, sa, omc, &bad);
      /* MBS with SRD+a: kappa sets the cell's relative kinetic energy after
       * the corrected collision to the drawn E_k */
      orc_sum K2s = sum_new(p);
      for (uint32_t j = b; j < e; ++j) {
        uint32_t i = perm[j];
        double du[3] = {v[i] - V[0], v[n + i] - V[1], v[2 * n + i] - V[2]};
        sum_add(&K2s, m * (du[0] * du[0] + du[1] * du[1] + du[2] * du[2]), &bad);
      }
      double K2 = sum_val(&K2s);
      kappa = 1.0;
      if (have_ek && K2 > 0.0) kappa = sqrt((2.0 * Ek) / K2);
      Kpost = 0.0;
      for (uint32_t j = b; j < e; ++j) {
        uint32_t i = perm[j];
        for (int k = 0; k < 3; ++k) {
          double du = kappa * (v[k * n + i] - V[k]);
          v[k * n + i] = V[k] + du;
          Kpost = Kpost + m * du * du;
        }
      }
    }
    if (le) {
      for (uint32_t j = b; j < e; ++j) {
        uint32_t i = perm[j];
        int side = le_side(p, x[2 * n + i], s[2]);
        if (side < 0) v[i] = v[i] + p->le_u;
        if (side > 0) v[i] = v[i] - p->le_u;
      }
    }
    if (co) {
      co[ORC_C_NX] = ax[0];
      co[ORC_C_NY] = ax[1];
      co[ORC_C_NZ] = ax[2];
      co[ORC_C_KAPPA] = kappa;
      co[ORC_C_KPOST] = Kpost;
    }
  }

  free(v0);
  if (xa != x) free(xa);
  if (p->g[0] != 0.0 || p->g[1] != 0.0 || p->g[2] != 0.0) {
    for (int k = 0; k < 3; ++k) {
      double gh = p->g[k] * p->h;
      for (int64_t i = 0; i < n; ++i) v[k * n + i] = v[k * n + i] + gh;
    }
  }
  return bad ? -3 : 0;
}

/* Sec. III.B.3: particles stored in cell order (here: this step's order). */
void orc_reorder(int64_t n, double* x, double* v, const uint32_t* perm) {
  double* tmp = (double*)malloc((size_t)n * sizeof(double));
  double* arrs[6] = {x, x + n, x + 2 * n, v, v + n, v + 2 * n};
  for (int a = 0; a < 6; ++a) {
    for (int64_t j = 0; j < n; ++j) tmp[j] = arrs[a][perm[j]];
    memcpy(arrs[a], tmp, (size_t)n * sizeof(double));
  }
  free(tmp);
}

int orc_step(const orc_params* p, uint64_t t, int64_t n, double* x, double* v, int32_t reorder,
             uint32_t* key_out, uint32_t* perm_out, uint32_t* offset_out) {
  int64_t ncell = orc_ncells(p);
  uint32_t* key = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  uint32_t* perm = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  uint32_t* offset = (uint32_t*)malloc(((size_t)ncell + 1) * sizeof(uint32_t));
  orc_stream(p, t, n, x, v);
  int rc = orc_keys(p, t, n, x, key);
  if (rc == 0) {
    orc_sort(n, key, ncell, perm, offset);
    rc = orc_collide(p, t, n, x, v, perm, offset, ncell, NULL);
    if (key_out) memcpy(key_out, key, (size_t)n * sizeof(uint32_t));
    if (perm_out) memcpy(perm_out, perm, (size_t)n * sizeof(uint32_t));
    if (offset_out) memcpy(offset_out, offset, ((size_t)ncell + 1) * sizeof(uint32_t));
    if (reorder) orc_reorder(n, x, v, perm);
  }
  free(key);
  free(perm);
  free(offset);
  return rc;
}

/* Neumaier's compensated summation. */
typedef struct {
  double s, c;
} nsum;
static void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

void orc_observables(const orc_params* p, int64_t n, const double* v, double out[6]) {
  const double m = p->mass;
  nsum P[3] = {{0, 0}, {0, 0}, {0, 0}}, E = {0, 0}, K = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    double e = 0.0;
    for (int k = 0; k < 3; ++k) {
      double vk = v[k * n + i];
      nadd(&P[k], m * vk);
      e = e + vk * vk;
    }
    nadd(&E, 0.5 * m * e);
  }
  double M = (double)n * m;
  double V[3] = {nval(&P[0]) / M, nval(&P[1]) / M, nval(&P[2]) / M};
  for (int64_t i = 0; i < n; ++i) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double d = v[k * n + i] - V[k];
      d2 = d2 + d * d;
    }
    nadd(&K, m * d2);
  }
  out[0] = nval(&P[0]);
  out[1] = nval(&P[1]);
  out[2] = nval(&P[2]);
  out[3] = nval(&E);
  out[4] = n > 1 ? nval(&K) / (3.0 * (double)(n - 1)) : 0.0;
  out[5] = (double)n;
}
