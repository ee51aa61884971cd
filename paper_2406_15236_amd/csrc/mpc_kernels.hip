// mpc_kernels.hip -- gfx950 kernels of the MPC-SRD step (arXiv:2406.15236, Sec. II).
//
// One step t on the device (steady state):
//   scan    : offset = exclusive prefix of hist (particles per cell of step t),
//             per-cell random draws; hist is zeroed for the next count
//   scatter : perm[offset[key] + rank] = i (each particle already holds its
//             rank inside its cell)
//   collide : per tile of cells: gather the cell segments through perm, order
//             each segment by logical index in LDS, stream (Eq. 1), sum the
//             cells one thread per cell, rotate (Eq. 2) + scale with the draws,
//             stream + bin for step t+1, and write the state into the other
//             buffer, each tile pass grouped by next-step cell; the next
//             step's counts and ranks come from one atomic per (pass, cell).
//   advance : t += 1, flip the buffers.
// The prologue kernel computes key/hist/rank of step t when the state was set
// from outside.  Every kernel reads the step index and buffer from Ctrl, so a
// captured graph of one step can be replayed.
#include <math.h>

#include "mpc_internal.h"
#include "philox_dev.h"

namespace mpc {

// Box parameters and tile/control tables are read-only while a kernel runs.
// Reading them through the constant address space lets the compiler use
// scalar loads that later global stores cannot clobber (otherwise every use
// after a store becomes a per-lane reload from memory).
#define MPC_AS4 __attribute__((address_space(4)))
using BoxRef = const MPC_AS4 BoxDev&;
template <typename T>
__device__ __forceinline__ const MPC_AS4 T* as_const(const T* p) {
  return (const MPC_AS4 T*)p;
}
__device__ __forceinline__ Tile load_tile(const Tile* p, uint32_t i) {
  const MPC_AS4 Tile& r = as_const(p)[i];
  Tile t;
  t.c0 = r.c0;
  t.nc = r.nc;
  t.box = r.box;
  t.x0 = r.x0;
  t.y0 = r.y0;
  t.z0 = r.z0;
  return t;
}
__device__ __forceinline__ PBlock load_pblock(const PBlock* p, uint32_t i) {
  const MPC_AS4 PBlock& r = as_const(p)[i];
  PBlock b;
  b.box = r.box;
  b.p0 = r.p0;
  return b;
}

// ---------------------------------------------------------------------------
// Random draws of the method
// ---------------------------------------------------------------------------
__device__ __forceinline__ Words4 draw(BoxRef B, uint32_t j, uint32_t id, uint64_t t,
                                       uint32_t tag) {
  return philox10(j, id, (uint32_t)t, tag, B.key_lo, B.key_hi);
}

// Lattice shift of step t: s_k = u24(w_k) - 1/2 (exact 2^-24 grid).
__device__ __forceinline__ void shift_of(BoxRef B, uint64_t t, double s[3]) {
  const Words4 w = draw(B, 0, 0, t, kTagShift);
  s[0] = u24_of(w.w[0]) - 0.5;
  s[1] = u24_of(w.w[1]) - 0.5;
  s[2] = u24_of(w.w[2]) - 0.5;
}

// Uniform random axis on the unit sphere: z = 1 - 2 u1, phi = 2 pi u2.
__device__ __forceinline__ void axis_of(BoxRef B, uint64_t t, uint32_t key, double n[3]) {
  const Words4 w = draw(B, 0, key, t, kTagAxis);
  const double u1 = u53_of(w.w[0], w.w[1]);
  const double u2 = u53_of(w.w[2], w.w[3]);
  const double z = 1.0 - 2.0 * u1;
  const double r = sqrt(1.0 - z * z);
  const double phi = kTwoPi * u2;
  double sp, cp;
  sincos(phi, &sp, &cp);
  n[0] = r * cp;
  n[1] = r * sp;
  n[2] = z;
}

// Gamma(shape, 1) by Marsaglia-Tsang; attempt j uses THERMO draw j
// (Box-Muller cosine branch from words 0,1; acceptance uniform from 2,3).
// Returns false if 64 attempts were rejected.
__device__ __forceinline__ bool gamma_of(BoxRef B, uint64_t t, uint32_t key, double shape,
                                      double* out) {
  const double d = shape - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
#pragma unroll 1
  for (uint32_t j = 0; j < 64; ++j) {
    const Words4 w = draw(B, j, key, t, kTagThermo);
    const double u1 = u32_open_of(w.w[0]);
    const double u2 = (double)w.w[1] * 0x1p-32;
    const double z = sqrt(-2.0 * log(u1)) * cos(kTwoPi * u2);
    double vv = 1.0 + c * z;
    if (vv <= 0.0) continue;
    vv = vv * vv * vv;
    const double u = u53_open_of(w.w[2], w.w[3]);
    const double lhs = log(u);
    const double rhs = 0.5 * z * z + d - d * vv + d * log(vv);
    if (lhs < rhs) {
      *out = d * vv;
      return true;
    }
  }
  return false;
}

// Phantom particles of a wall-cut cell: Poisson(<N_c> f_w) count by inversion
// on draw 0, truncated at 127.
__device__ __forceinline__ int phantom_count(BoxRef B, uint64_t t, uint32_t key, double fw) {
  const double lam = B.density * fw;
  const Words4 w = draw(B, 0, key, t, kTagPhantom);
  const double u = u53_of(w.w[0], w.w[1]);
  int k = 0;
  double pk = exp(-lam);
  double F = pk;
#pragma unroll 1
  while (u >= F && k < 127) {
    k += 1;
    pk = pk * lam / (double)k;
    F = F + pk;
  }
  return k;
}

// Normal number m of a cell's phantom stream (draw 1 + m/4; Box-Muller pair
// (m%4)/2; cosine for even m, sine for odd m).  `cache` keeps the last draw.
struct PhantomCache {
  uint32_t j;
  Words4 w;
};
__device__ __forceinline__ double phantom_normal(BoxRef B, uint64_t t, uint32_t key,
                                                 uint32_t m, PhantomCache& pc) {
  const uint32_t j = 1 + m / 4;
  if (pc.j != j) {
    pc.w = draw(B, j, key, t, kTagPhantom);
    pc.j = j;
  }
  const uint32_t pr = (m % 4) / 2;
  const double r = sqrt(-2.0 * log(u32_open_of(pc.w.w[2 * pr])));
  const double th = kTwoPi * ((double)pc.w.w[2 * pr + 1] * 0x1p-32);
  return (m % 2 == 0) ? r * cos(th) : r * sin(th);
}

// Wall volume fraction of shifted z layer cz (layer spans [cz - sz, cz + 1 - sz)).
__device__ __forceinline__ double wall_fraction(double sz, int cz, int H) {
  if (sz >= 0.0) {
    if (cz == 0) return sz;
    if (cz == H) return 1.0 - sz;
  } else {
    if (cz == -1) return 1.0 + sz;
    if (cz == H - 1) return -sz;
  }
  return 0.0;
}

// ---------------------------------------------------------------------------
// Storage forms
// ---------------------------------------------------------------------------
// Periodic wrap into [0, L): one image shift (selects), then the rare cases
// (rounding onto L, far outside, non-finite) on a cold path.
__device__ __noinline__ double wrap64_rare(double x, double L) {
  if (x == L) return 0.0;
  if (isfinite(x)) {
    x = x - L * floor(x / L);
    if (x >= L || x < 0.0) x = 0.0;
  }
  return x;
}
__device__ __forceinline__ double wrap64(double x, double L) {
  const double lo = x + L, hi = x - L;
  x = x < 0.0 ? lo : (x >= L ? hi : x);
  if (__builtin_expect(!(x >= 0.0 && x < L), 0)) x = wrap64_rare(x, L);
  return x;
}

__device__ __noinline__ float wrap32_rare(float x, float L) {
  if (x == L) return 0.0f;
  if (isfinite(x)) {
    x = x - L * floorf(x / L);
    if (x >= L || x < 0.0f) x = 0.0f;
  }
  return x;
}
__device__ __forceinline__ float wrap32(float x, float L) {
  const float lo = x + L, hi = x - L;
  x = x < 0.0f ? lo : (x >= L ? hi : x);
  if (__builtin_expect(!(x >= 0.0f && x < L), 0)) x = wrap32_rare(x, L);
  return x;
}

// Lees-Edwards shear of a periodic box (Sec. II, boundary conditions): at
// time tau = t_end h the image above the box (z + L_z) is displaced by
// d = (U tau) mod L_x along x and moves with U.  A particle through a z face
// re-enters displaced by -/+ d with v_x -/+ U; a collision cell across a z
// face is formed with the image on the other side, in that image's frame.
__device__ __forceinline__ double le_offset(BoxRef B, uint64_t t_end) {
  const double d = B.leu * ((double)t_end * B.h);
  return d - B.Ld[0] * floor(d / B.Ld[0]);
}

// Eq.(1) in FP64 with periodic x, y and (walls) time-reversed bounce-back in z;
// dle: Lees-Edwards offset at the end of this streaming.
template <bool W>
__device__ __forceinline__ void stream_f64(double (&x)[3], double (&v)[3], BoxRef B,
                                           double dle, bool le) {
  double xe = fma(B.h, v[0], x[0]);
  double ye = fma(B.h, v[1], x[1]);
  double ze = fma(B.h, v[2], x[2]);
  if (W) {
    const double H = B.Ld[2];
    const bool lo = ze < 0.0, hi = ze > H;
    if (lo || hi) {
      const double zw = lo ? 0.0 : H;
      const double tr2 = 2.0 * ((ze - zw) / v[2]);
      if (B.slip) {  // specular reflection
        ze = ze - tr2 * v[2];
      } else {       // bounce-back in the frame of the (moving) wall
        const double uw = lo ? -B.uw : B.uw;
        xe = xe - tr2 * (v[0] - uw);
        ye = ye - tr2 * v[1];
        ze = ze - tr2 * v[2];
        v[0] = 2.0 * uw - v[0];
        v[1] = -v[1];
      }
      if (ze < 0.0) ze = 0.0;
      if (ze > H) ze = H;
      v[2] = -v[2];
    }
  } else {
    if (le && (ze >= B.Ld[2] || ze < 0.0)) {
      if (ze >= B.Ld[2]) {
        xe = xe - dle;
        v[0] = v[0] - B.leu;
      } else {
        xe = xe + dle;
        v[0] = v[0] + B.leu;
      }
    }
    ze = wrap64(ze, B.Ld[2]);
  }
  x[0] = wrap64(xe, B.Ld[0]);
  x[1] = wrap64(ye, B.Ld[1]);
  x[2] = ze;
}

template <bool W>
__device__ __forceinline__ void stream_f32(float (&x)[3], float (&v)[3], BoxRef B, double dle,
                                           bool le) {
  float xe = fmaf(B.hf, v[0], x[0]);
  float ye = fmaf(B.hf, v[1], x[1]);
  float ze = fmaf(B.hf, v[2], x[2]);
  if (W) {
    const float H = B.Lf[2];
    const bool lo = ze < 0.0f, hi = ze > H;
    if (lo || hi) {
      const float zw = lo ? 0.0f : H;
      const float tr2 = 2.0f * ((ze - zw) / v[2]);
      if (B.slip) {
        ze = ze - tr2 * v[2];
      } else {
        const float uw = lo ? -B.uwf : B.uwf;
        xe = xe - tr2 * (v[0] - uw);
        ye = ye - tr2 * v[1];
        ze = ze - tr2 * v[2];
        v[0] = 2.0f * uw - v[0];
        v[1] = -v[1];
      }
      if (ze < 0.0f) ze = 0.0f;
      if (ze > H) ze = H;
      v[2] = -v[2];
    }
  } else {
    if (le && (ze >= B.Lf[2] || ze < 0.0f)) {
      if (ze >= B.Lf[2]) {
        xe = xe - (float)dle;
        v[0] = v[0] - B.leuf;
      } else {
        xe = xe + (float)dle;
        v[0] = v[0] + B.leuf;
      }
    }
    ze = wrap32(ze, B.Lf[2]);
  }
  x[0] = wrap32(xe, B.Lf[0]);
  x[1] = wrap32(ye, B.Lf[1]);
  x[2] = ze;
}

// Split form: unshifted cell (packed) + offset in [0, 1) per axis.
__device__ __forceinline__ void split_decode(uint32_t cell, int (&c)[3]) {
  c[0] = (int)(cell & ((1u << kSplitXBits) - 1));
  c[1] = (int)((cell >> kSplitXBits) & ((1u << kSplitYBits) - 1));
  c[2] = (int)(cell >> (kSplitXBits + kSplitYBits));
}
__device__ __forceinline__ uint32_t split_encode(const int (&c)[3]) {
  return (uint32_t)c[0] | ((uint32_t)c[1] << kSplitXBits) |
         ((uint32_t)c[2] << (kSplitXBits + kSplitYBits));
}
__device__ __noinline__ int wrap_cell_rare(int c, int L) { return ((c % L) + L) % L; }
__device__ __forceinline__ int wrap_cell(int c, int L) {
  c = c < 0 ? c + L : (c >= L ? c - L : c);
  if (__builtin_expect(c < 0 || c >= L, 0)) c = wrap_cell_rare(c, L);
  return c;
}
// FP64 value -> (cell, offset) with the offset rounded to FP32.
__device__ __forceinline__ void split_from_double(double xd, int& c, float& o) {
  const double fl = floor(xd);
  c = (int)fl;
  o = (float)(xd - fl);
  if (o >= 1.0f) {
    o = 0.0f;
    c += 1;
  }
}

template <bool W>
__device__ __forceinline__ void stream_split(uint32_t& cell, float (&o)[3], float (&v)[3],
                                             BoxRef B, double dle, bool le) {
  int c[3];
  split_decode(cell, c);
  int cn[3];
  float on[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float y = fmaf(B.hf, v[k], o[k]);
    float fl = floorf(y);
    y = y - fl;
    if (y == 1.0f) {
      y = 0.0f;
      fl += 1.0f;
    }
    on[k] = y;
    cn[k] = c[k] + (int)fl;
  }
  if (W) {
    const int H = B.L[2];
    const bool out = cn[2] < 0 || cn[2] > H || (cn[2] == H && on[2] > 0.0f) ||
                     !isfinite(on[2]);
    if (out) {
      // crossing particle: the bounce is done in FP64 from the exact position
      double xd[3], vd[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xd[k] = (double)c[k] + (double)o[k];
        vd[k] = (double)v[k];
      }
      double xe[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xe[k] = fma(B.h, vd[k], xd[k]);
      const double Hd = B.Ld[2];
      if (xe[2] < 0.0 || xe[2] > Hd) {
        const bool lo = xe[2] < 0.0;
        const double zw = lo ? 0.0 : Hd;
        const double tr2 = 2.0 * ((xe[2] - zw) / vd[2]);
        if (B.slip) {
          xe[2] = xe[2] - tr2 * vd[2];
        } else {
          const double uw = lo ? -B.uw : B.uw;
          xe[0] = xe[0] - tr2 * (vd[0] - uw);
          xe[1] = xe[1] - tr2 * vd[1];
          xe[2] = xe[2] - tr2 * vd[2];
          v[0] = (float)(2.0 * uw - vd[0]);
          v[1] = -v[1];
        }
        if (xe[2] < 0.0) xe[2] = 0.0;
        if (xe[2] > Hd) xe[2] = Hd;
        v[2] = -v[2];
      }
      xe[0] = wrap64(xe[0], B.Ld[0]);
      xe[1] = wrap64(xe[1], B.Ld[1]);
#pragma unroll
      for (int k = 0; k < 3; ++k) split_from_double(xe[k], cn[k], on[k]);
    }
  } else {
    if (le && (cn[2] >= B.L[2] || cn[2] < 0)) {
      // through a sheared face: x -/+ d in FP64, v_x -/+ U
      const bool up = cn[2] >= B.L[2];
      double xd = (double)cn[0] + (double)on[0];
      xd = wrap64(up ? xd - dle : xd + dle, B.Ld[0]);
      split_from_double(xd, cn[0], on[0]);
      v[0] = (float)(up ? (double)v[0] - B.leu : (double)v[0] + B.leu);
    }
    cn[2] = wrap_cell(cn[2], B.L[2]);
  }
  cn[0] = wrap_cell(cn[0], B.L[0]);
  cn[1] = wrap_cell(cn[1], B.L[1]);
  o[0] = on[0];
  o[1] = on[1];
  o[2] = on[2];
  cell = split_encode(cn);
}

// c + L if c < 0, c - L if c >= L (c within one period of [0, L)); branch-free.
__device__ __forceinline__ int wrap1(int c, int L) {
  c += L & -(int)(c < 0);
  c -= L & -(int)(c >= L);
  return c;
}

// Shifted cell coordinates c_k = floor(x_k + s_k) of a position given as
// integer part ci_k plus fraction xf_k in double (exact), with periodic wrap
// (walls: z becomes the layer index c_z + 1 in [0, H+1]).  Invalid -> err.
template <bool W>
__device__ __forceinline__ bool coords_of(const int (&ci)[3], const double (&xf)[3],
                                          const double (&s)[3], BoxRef B, int (&c)[3],
                                          uint32_t& err, double dle, bool le) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double y = xf[k] + s[k];
    const bool in = y >= -2.0 && y < B.Ld[k] + 2.0;
    ok = ok && in;
    c[k] = ci[k] + (int)floor(in ? y : 0.0);
  }
  if (!W && le && (c[2] < 0 || c[2] >= B.L[2])) {
    // Lees-Edwards: a cell across a z face is formed with the image on the
    // other side (x -/+ d of the collision time)
    const double xi = c[2] >= B.L[2] ? xf[0] - dle : xf[0] + dle;
    c[0] = wrap1(ci[0] + (int)floor(xi + s[0]), B.L[0]);
  }
  c[0] = wrap1(c[0], B.L[0]);
  c[1] = wrap1(c[1], B.L[1]);
  if (W) {
    c[2] += 1;
  } else {
    c[2] = wrap1(c[2], B.L[2]);
  }
  ok = ok && (unsigned)c[0] < (unsigned)B.L[0] && (unsigned)c[1] < (unsigned)B.L[1] &&
       (unsigned)c[2] < (unsigned)B.nlz;
  if (__builtin_expect(!ok, 0)) {
    err |= kErrKey;
    c[0] = c[1] = c[2] = 0;
  }
  return ok;
}

// Split form: c_k = cell_k + floor(o_k + s_k) with the sum in FP32, which
// gives the exact floor: o is an FP32 offset in [0, 1) and s lies on the
// 2^-24 grid in [-1/2, 1/2), so o + s is exact whenever it is below 1 or near
// 0 (Sterbenz), and a sum of at least 1 stays below 2.
template <bool W>
__device__ __forceinline__ bool coords_split(const int (&ci)[3], const float (&o)[3],
                                             const double (&s)[3], BoxRef B, int (&c)[3],
                                             uint32_t& err) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float y = o[k] + (float)s[k];
    const bool in = y >= -2.0f && y < 2.0f;
    ok = ok && in;
    c[k] = ci[k] + (int)floorf(in ? y : 0.0f);
  }
  c[0] = wrap1(c[0], B.L[0]);
  c[1] = wrap1(c[1], B.L[1]);
  if (W) {
    c[2] += 1;
  } else {
    c[2] = wrap1(c[2], B.L[2]);
  }
  ok = ok && (unsigned)c[0] < (unsigned)B.L[0] && (unsigned)c[1] < (unsigned)B.L[1] &&
       (unsigned)c[2] < (unsigned)B.nlz;
  if (__builtin_expect(!ok, 0)) {
    err |= kErrKey;
    c[0] = c[1] = c[2] = 0;
  }
  return ok;
}

__device__ __forceinline__ uint32_t linear_key(const int (&c)[3], BoxRef B) {
  return (uint32_t)((c[2] * B.L[1] + c[1]) * B.L[0] + c[0]);
}

template <bool W>
__device__ __forceinline__ uint32_t key_of(const int (&ci)[3], const double (&xf)[3],
                                           const double (&s)[3], BoxRef B, uint32_t& err,
                                           double dle, bool le) {
  int c[3];
  coords_of<W>(ci, xf, s, B, c, err, dle, le);
  return linear_key(c, B);
}

// Per-form particle access.  P = position type, V = velocity type,
// Vs = LDS velocity type, R = rotation arithmetic type.
template <int F>
struct Form;

template <>
struct Form<kFormF64> {
  struct P {
    double x[3];
  };
  struct Vv {
    double v[3];
  };
  using Vs = double;
  using Xs = double;
  static constexpr bool kHasCell = false;
  __device__ static void to_lds(const P& p, Xs* x0, Xs* x1, Xs* x2, uint32_t*, uint32_t q) {
    x0[q] = p.x[0];
    x1[q] = p.x[1];
    x2[q] = p.x[2];
  }
  __device__ static void from_lds(P& p, const Xs* x0, const Xs* x1, const Xs* x2,
                                  const uint32_t*, uint32_t q) {
    p.x[0] = x0[q];
    p.x[1] = x1[q];
    p.x[2] = x2[q];
  }
  // record: three 16-byte words (x0 x1 | x2 v0 | v1 v2)
  __device__ static void load(const StatePtrs& S, uint32_t i, P& p, Vv& v) {
    const double2* r = (const double2*)S.rec + 3 * (size_t)i;
    const double2 a = r[0], b = r[1], c = r[2];
    p.x[0] = a.x;
    p.x[1] = a.y;
    p.x[2] = b.x;
    v.v[0] = b.y;
    v.v[1] = c.x;
    v.v[2] = c.y;
  }
  __device__ static void load_all(const StatePtrs& S, uint32_t i, P& p, Vv& v, uint32_t& id) {
    load(S, i, p, v);
    id = S.id[i];
  }
  __device__ static void store_all(const StatePtrs& S, uint32_t j, const P& p, const Vv& v,
                                   uint32_t id) {
    double2* r = (double2*)S.rec + 3 * (size_t)j;
    r[0] = make_double2(p.x[0], p.x[1]);
    r[1] = make_double2(p.x[2], v.v[0]);
    r[2] = make_double2(v.v[1], v.v[2]);
    S.id[j] = id;
  }
  template <bool W>
  __device__ static void stream(P& p, Vv& v, BoxRef B, double dle, bool le) {
    stream_f64<W>(p.x, v.v, B, dle, le);
  }
  template <bool W>
  __device__ static uint32_t key(const P& p, const double (&s)[3], BoxRef B,
                                 uint32_t& err, double dle, bool le) {
    const int ci[3] = {0, 0, 0};
    const double xf[3] = {p.x[0], p.x[1], p.x[2]};
    return key_of<W>(ci, xf, s, B, err, dle, le);
  }
  template <bool W>
  __device__ static void coords(const P& p, const double (&s)[3], BoxRef B, int (&c)[3],
                                uint32_t& err, double dle, bool le) {
    const int ci[3] = {0, 0, 0};
    const double xf[3] = {p.x[0], p.x[1], p.x[2]};
    coords_of<W>(ci, xf, s, B, c, err, dle, le);
  }
  // Lees-Edwards side of the collision cell: +1 below the lower z face,
  // -1 above the upper one, else 0
  __device__ static int le_side(const P& p, double sz, BoxRef B) {
    const double cz = floor(p.x[2] + sz);
    return cz < 0.0 ? 1 : (cz >= B.Ld[2] ? -1 : 0);
  }
};

template <>
struct Form<kFormF32> {
  struct P {
    float x[3];
  };
  struct Vv {
    float v[3];
  };
  using Vs = float;
  using Xs = float;
  static constexpr bool kHasCell = false;
  __device__ static void to_lds(const P& p, Xs* x0, Xs* x1, Xs* x2, uint32_t*, uint32_t q) {
    x0[q] = p.x[0];
    x1[q] = p.x[1];
    x2[q] = p.x[2];
  }
  __device__ static void from_lds(P& p, const Xs* x0, const Xs* x1, const Xs* x2,
                                  const uint32_t*, uint32_t q) {
    p.x[0] = x0[q];
    p.x[1] = x1[q];
    p.x[2] = x2[q];
  }
  // record: three 8-byte words (x0 x1 | x2 v0 | v1 v2)
  __device__ static void load(const StatePtrs& S, uint32_t i, P& p, Vv& v) {
    const float2* r = (const float2*)S.rec + 3 * (size_t)i;
    const float2 a = r[0], b = r[1], c = r[2];
    p.x[0] = a.x;
    p.x[1] = a.y;
    p.x[2] = b.x;
    v.v[0] = b.y;
    v.v[1] = c.x;
    v.v[2] = c.y;
  }
  __device__ static void load_all(const StatePtrs& S, uint32_t i, P& p, Vv& v, uint32_t& id) {
    load(S, i, p, v);
    id = S.id[i];
  }
  __device__ static void store_all(const StatePtrs& S, uint32_t j, const P& p, const Vv& v,
                                   uint32_t id) {
    float2* r = (float2*)S.rec + 3 * (size_t)j;
    r[0] = make_float2(p.x[0], p.x[1]);
    r[1] = make_float2(p.x[2], v.v[0]);
    r[2] = make_float2(v.v[1], v.v[2]);
    S.id[j] = id;
  }
  template <bool W>
  __device__ static void stream(P& p, Vv& v, BoxRef B, double dle, bool le) {
    stream_f32<W>(p.x, v.v, B, dle, le);
  }
  template <bool W>
  __device__ static uint32_t key(const P& p, const double (&s)[3], BoxRef B,
                                 uint32_t& err, double dle, bool le) {
    const int ci[3] = {0, 0, 0};
    const double xf[3] = {(double)p.x[0], (double)p.x[1], (double)p.x[2]};
    return key_of<W>(ci, xf, s, B, err, dle, le);
  }
  template <bool W>
  __device__ static void coords(const P& p, const double (&s)[3], BoxRef B, int (&c)[3],
                                uint32_t& err, double dle, bool le) {
    const int ci[3] = {0, 0, 0};
    const double xf[3] = {(double)p.x[0], (double)p.x[1], (double)p.x[2]};
    coords_of<W>(ci, xf, s, B, c, err, dle, le);
  }
  __device__ static int le_side(const P& p, double sz, BoxRef B) {
    const double cz = floor((double)p.x[2] + sz);
    return cz < 0.0 ? 1 : (cz >= B.Ld[2] ? -1 : 0);
  }
};

template <>
struct Form<kFormSplit> {
  struct P {
    uint32_t cell;
    float o[3];
  };
  struct Vv {
    float v[3];
  };
  using Vs = float;
  using Xs = float;
  static constexpr bool kHasCell = true;
  __device__ static void to_lds(const P& p, Xs* x0, Xs* x1, Xs* x2, uint32_t* c, uint32_t q) {
    x0[q] = p.o[0];
    x1[q] = p.o[1];
    x2[q] = p.o[2];
    c[q] = p.cell;
  }
  __device__ static void from_lds(P& p, const Xs* x0, const Xs* x1, const Xs* x2,
                                  const uint32_t* c, uint32_t q) {
    p.o[0] = x0[q];
    p.o[1] = x1[q];
    p.o[2] = x2[q];
    p.cell = c[q];
  }
  // record: two 16-byte words (cell o0 o1 o2 | v0 v1 v2 id).  The gather
  // reads the id word with a load of its own after the 28 bytes of state
  // (measured 8 % faster for the collide than one 16-byte load of v and id).
  __device__ static void load(const StatePtrs& S, uint32_t i, P& p, Vv& v) {
    const uint4* r = (const uint4*)S.rec + 2 * (size_t)i;
    const uint4 a = r[0];
    const uint32_t* w = (const uint32_t*)(r + 1);
    p.cell = a.x;
    p.o[0] = __uint_as_float(a.y);
    p.o[1] = __uint_as_float(a.z);
    p.o[2] = __uint_as_float(a.w);
    v.v[0] = __uint_as_float(w[0]);
    v.v[1] = __uint_as_float(w[1]);
    v.v[2] = __uint_as_float(w[2]);
  }
  __device__ static void load_all(const StatePtrs& S, uint32_t i, P& p, Vv& v, uint32_t& id) {
    load(S, i, p, v);
    id = S.id[(size_t)i * (sizeof(RecSplit) / 4)];
  }
  __device__ static void store_all(const StatePtrs& S, uint32_t j, const P& p, const Vv& v,
                                   uint32_t id) {
    uint4* r = (uint4*)S.rec + 2 * (size_t)j;
    r[0] = make_uint4(p.cell, __float_as_uint(p.o[0]), __float_as_uint(p.o[1]),
                      __float_as_uint(p.o[2]));
    r[1] = make_uint4(__float_as_uint(v.v[0]), __float_as_uint(v.v[1]), __float_as_uint(v.v[2]),
                      id);
  }
  template <bool W>
  __device__ static void stream(P& p, Vv& v, BoxRef B, double dle, bool le) {
    stream_split<W>(p.cell, p.o, v.v, B, dle, le);
  }
  template <bool W>
  __device__ static void coords(const P& p, const double (&s)[3], BoxRef B, int (&c)[3],
                                uint32_t& err, double dle, bool le) {
    int ci[3];
    split_decode(p.cell, ci);
    if (!le) {
      coords_split<W>(ci, p.o, s, B, c, err);
      return;
    }
    // Lees-Edwards: the image offset is applied in FP64
    const double xf[3] = {(double)p.o[0], (double)p.o[1], (double)p.o[2]};
    coords_of<W>(ci, xf, s, B, c, err, dle, le);
  }
  template <bool W>
  __device__ static uint32_t key(const P& p, const double (&s)[3], BoxRef B,
                                 uint32_t& err, double dle, bool le) {
    int c[3];
    coords<W>(p, s, B, c, err, dle, le);
    return linear_key(c, B);
  }
  __device__ static int le_side(const P& p, double sz, BoxRef B) {
    int ci[3];
    split_decode(p.cell, ci);
    const int cz = ci[2] + (int)floor((double)p.o[2] + sz);
    return cz < 0 ? 1 : (cz >= B.L[2] ? -1 : 0);
  }
};

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

__global__ void k_set_ctrl(Ctrl* c, uint64_t step, uint32_t cur, int32_t reorder, int clear_err) {
  c->step = step;
  c->cur = cur;
  c->reorder = reorder;
  if (clear_err) c->err = 0u;
}

__global__ void k_advance(Ctrl* c) {
  c->cur ^= 1u;
  c->step = c->step + 1;
}

// hist[c] += 1 for every active lane, one atomic per distinct key in the
// wavefront; returns the lane's rank among all particles counted for c (the
// old count of its run's leader plus its place in the run).
__device__ __forceinline__ uint32_t wave_hist_rank(uint32_t* hist, uint32_t c, bool active) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t pending = __ballot(active);
  uint64_t mine = 0;
  while (pending) {
    const int lead = __ffsll((unsigned long long)pending) - 1;
    const uint32_t lc = (uint32_t)__builtin_amdgcn_readlane((int)c, lead);
    const uint64_t same = __ballot(active && c == lc) & pending;
    if (active && c == lc) mine = same;
    pending &= ~same;
  }
  const uint32_t before = (uint32_t)__popcll(mine & lt_mask);
  uint32_t old = 0;
  if (active && before == 0) old = atomicAdd(&hist[c], (uint32_t)__popcll(mine));
  const int lead_lane = active ? (__ffsll((unsigned long long)mine) - 1) : (int)lane;
  old = __shfl(old, lead_lane, 64);
  return old + before;
}

// Prologue: key and histogram of step t from the current state.
template <int F, bool W>
__global__ __launch_bounds__(kThreads) void k_key_hist(Dev d) {
  using Fm = Form<F>;
  __shared__ double s_sh[3];
  const PBlock pb = load_pblock(d.pblocks, blockIdx.x);
  BoxRef B = as_const(d.boxes)[pb.box];
  const uint64_t t = d.ctrl->step;
  const StatePtrs S = d.S[d.ctrl->cur];
  if (threadIdx.x == 0) {
    double s[3];
    shift_of(B, t, s);
    s_sh[0] = s[0];
    s_sh[1] = s[1];
    s_sh[2] = s[2];
  }
  __syncthreads();
  const double s[3] = {s_sh[0], s_sh[1], s_sh[2]};
  const uint32_t pend = B.pbase + B.np;
  uint32_t err = 0;
#pragma unroll
  for (int k = 0; k < kPartBlock / kThreads; ++k) {
    const uint32_t i = pb.p0 + k * kThreads + threadIdx.x;
    uint32_t key = 0;
    if (i < pend) {
      typename Fm::P p;
      typename Fm::Vv v;
      Fm::load(S, i, p, v);
      const double dle = W ? 0.0 : le_offset(B, t + 1);
      Fm::template stream<W>(p, v, B, dle, !W && B.le);
      key = B.cbase + Fm::template key<W>(p, s, B, err, dle, !W && B.le);
      d.key[i] = key;
    }
    const uint32_t rk = wave_hist_rank(d.hist, key, i < pend);
    if (i < pend) d.rank[i] = (uint16_t)min(rk, 0xffffu);
  }
  if (err) atomicOr(&d.ctrl->err, err);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of hist -> offset (reduce, top, down-sweep)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int dlt = 1; dlt < 64; dlt <<= 1) {
    const uint32_t y = __shfl_up(x, dlt, 64);
    if (lane >= dlt) x += y;
  }
  return x;
}

// Exclusive block scan of one value per thread; returns the block total too.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_w,
                                                         uint32_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const uint32_t inc = wave_inclusive_scan(x);
  if (lane == 63) s_w[wid] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t sw = s_w[w];
    if (w < wid) pre += sw;
    tot += sw;
  }
  total = tot;
  __syncthreads();
  return pre + inc - x;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ blk) {
  __shared__ uint32_t s_w[kThreads / 64];
  const uint4* h4 = (const uint4*)(hist + (uint64_t)blockIdx.x * kScanBlock);
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems / 4; ++k) {
    const uint4 q = h4[k * kThreads + threadIdx.x];
    sum += q.x + q.y + q.z + q.w;
  }
  uint32_t total;
  block_exclusive_scan(sum, s_w, total);
  if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// One workgroup of 1024 threads scans all block totals in place (exclusive).
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ blk, uint32_t nblk) {
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nblk; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t x = i < nblk ? blk[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(x, s_w, total);
    const uint32_t carry = s_carry;
    if (i < nblk) blk[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + total;
    __syncthreads();
  }
}

// Box that owns global cell c (boxes are stored in ascending cbase).
__device__ __forceinline__ uint32_t box_of_cell(const BoxDev* boxes, uint32_t nbox, uint32_t c) {
  uint32_t lo = 0, hi = nbox;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (as_const(boxes)[mid].cbase <= c) {
      lo = mid;
    } else {
      hi = mid;
    }
  }
  return lo;
}

// Random draws of one occupied cell for step t: the rotation axis and, with
// the thermostat, the target energy E_k = kT * Gamma(3 (n - 1) / 2), where n
// counts phantoms too (walls).  Ek = 0 means "no scaling".
template <bool W, bool M>
__device__ __forceinline__ void cell_draws(BoxRef B, uint64_t t, uint32_t lkey, uint32_t nf,
                                           double sz, CellDraw& out) {
  uint32_t ntot = nf;
  if (W && !B.slip) {
    const int cz = (int)(lkey / (uint32_t)(B.L[0] * B.L[1])) - 1;
    const double fw = wall_fraction(sz, cz, B.L[2]);
    if (fw > 0.0) ntot += (uint32_t)phantom_count(B, t, lkey, fw);
  }
  axis_of(B, t, lkey, out.n);
  out.Ek = 0.0;
  if (M && ntot >= 2) {
    double gv;
    if (gamma_of(B, t, lkey, 1.5 * (double)(ntot - 1), &gv)) out.Ek = B.kT * gv;
  }
}

// Each thread owns kScanItems consecutive cells: offsets, then the cell draws
// of its occupied cells (all lanes busy: one thread per 16 cells).
template <bool W, bool M>
__global__ __launch_bounds__(kThreads) void k_scan_down(Dev d, uint32_t nblk, uint32_t nbox,
                                                        uint32_t ctot) {
  __shared__ uint32_t s_w[kThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
  uint4* h4 = (uint4*)(d.hist + base);
  uint32_t v[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems / 4; ++k) {
    const uint4 q = h4[k];
    v[4 * k] = q.x;
    v[4 * k + 1] = q.y;
    v[4 * k + 2] = q.z;
    v[4 * k + 3] = q.w;
    h4[k] = make_uint4(0u, 0u, 0u, 0u);  // the next collide counts from zero
  }
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) sum += v[k];
  uint32_t total;
  uint32_t run = d.scan_blk[blockIdx.x] + block_exclusive_scan(sum, s_w, total);
  uint4* o4 = (uint4*)(d.offset + base);
#pragma unroll
  for (int k = 0; k < kScanItems / 4; ++k) {
    uint4 q;
    q.x = run;
    run += v[4 * k];
    q.y = run;
    run += v[4 * k + 1];
    q.z = run;
    run += v[4 * k + 2];
    q.w = run;
    run += v[4 * k + 3];
    o4[k] = q;
  }
  if (blockIdx.x == nblk - 1 && threadIdx.x == kThreads - 1)
    d.offset[(uint64_t)nblk * kScanBlock] = run;

  // per-cell draws for step t; the counts go through LDS so that consecutive
  // lanes draw (and store the 32-byte records of) consecutive cells
  __shared__ uint4 s_cnt[kScanBlock / 4];
#pragma unroll
  for (int k = 0; k < kScanItems / 4; ++k)
    s_cnt[threadIdx.x * (kScanItems / 4) + k] =
        make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  __syncthreads();
  const uint64_t blk0 = (uint64_t)blockIdx.x * kScanBlock;
  if (blk0 + threadIdx.x >= ctot) return;
  const uint32_t* cnt = (const uint32_t*)s_cnt;
  const uint64_t t = as_const(d.ctrl)->step;
  uint32_t b = box_of_cell(d.boxes, nbox, (uint32_t)(blk0 + threadIdx.x));
  double sz = 0.0;
  if (W) {
    double sh[3];
    shift_of(as_const(d.boxes)[b], t, sh);
    sz = sh[2];
  }
#pragma unroll 1
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t c = (uint32_t)(blk0 + (uint64_t)k * kThreads + threadIdx.x);
    if (c >= ctot) break;
    while (c >= as_const(d.boxes)[b].cbase + as_const(d.boxes)[b].nc) {
      ++b;
      if (W) {
        double sh[3];
        shift_of(as_const(d.boxes)[b], t, sh);
        sz = sh[2];
      }
    }
    const uint32_t nf = cnt[k * kThreads + threadIdx.x];
    if (nf == 0u) continue;
    BoxRef B = as_const(d.boxes)[b];
    CellDraw cd;
    cell_draws<W, M>(B, t, c - B.cbase, nf, sz, cd);
    d.draws[c] = cd;
  }
}

// ---------------------------------------------------------------------------
// Scatter: slot of each particle inside its cell segment (order inside a
// segment is arbitrary here and made canonical in collide).
// ---------------------------------------------------------------------------
// Phantom particles of the occupied cells of the two wall-cut layers of every
// box (one thread per cell of those layers): count, velocity sum and squared-
// speed sum (velocities N(0, kT/m) per component; rounded to FP32 for the
// split form), read by the collide's cell sums.
__global__ __launch_bounds__(kThreads) void k_phantom_sums(Dev d, uint32_t nbox, uint32_t wcells,
                                                           int round32) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= wcells) return;
  uint32_t lo = 0, hi = nbox;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (d.boxes[mid].wcbase <= i) {
      lo = mid;
    } else {
      hi = mid;
    }
  }
  BoxRef B = as_const(d.boxes)[lo];
  if (B.slip) return;  // slip walls carry no phantoms
  const uint64_t t = as_const(d.ctrl)->step;
  double sh[3];
  shift_of(B, t, sh);
  const uint32_t plane = (uint32_t)B.L[0] * (uint32_t)B.L[1];
  const uint32_t li = i - B.wcbase;
  const uint32_t top = li / plane;
  const int H = B.L[2];
  // key layer (c_z + 1) of the cut cells: c_z in {0, H} for s_z >= 0, {-1, H-1} else
  const int czk = sh[2] >= 0.0 ? (top ? H + 1 : 1) : (top ? H : 0);
  const uint32_t lkey = (uint32_t)czk * plane + (li - top * plane);
  const uint32_t c = B.cbase + lkey;
  if (d.offset[c + 1] == d.offset[c]) return;  // not occupied: no collision
  const double fw = wall_fraction(sh[2], czk - 1, H);
  if (!(fw > 0.0)) return;
  const int nph = phantom_count(B, t, lkey, fw);
  PhantomSums ps;
  ps.v[0] = ps.v[1] = ps.v[2] = 0.0;
  ps.v2 = 0.0;
  PhantomCache pc;
  pc.j = 0xffffffffu;
  // phantoms move with the wall that fills their part of the cell
  const double uw = top ? B.uw : -B.uw;
#pragma unroll 1
  for (int q = 0; q < nph; ++q) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double vp = B.sd * phantom_normal(B, t, lkey, 3 * q + k, pc);
      if (k == 0) vp = vp + uw;
      if (round32) vp = (double)(float)vp;
      ps.v[k] = ps.v[k] + vp;
      ps.v2 = ps.v2 + vp * vp;
    }
  }
  ps.n = (double)nph;
  ps.pad = 0.0;
  d.phs[c] = ps;
}

__global__ __launch_bounds__(kThreads) void k_scatter(const uint32_t* __restrict__ key,
                                                      const uint16_t* __restrict__ rank,
                                                      const uint32_t* __restrict__ offset,
                                                      uint32_t* __restrict__ perm, uint32_t n,
                                                      uint32_t ncell, Ctrl* ctrl) {
  // Every particle already holds its rank among the particles of its cell
  // (taken when the cell's count was accumulated): no atomics here.
  uint32_t bad = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = blockIdx.x * (kThreads * 4) + k * kThreads + threadIdx.x;
    if (i >= n) continue;
    const uint32_t c = key[i];
    if (c >= ncell) {
      bad = 1;
      continue;
    }
    const uint32_t slot = offset[c] + rank[i];
    if (slot >= offset[c + 1] || slot >= n) {
      bad = 1;
    } else {
      perm[slot] = i;
    }
  }
  if (bad) atomicOr(&ctrl->err, kErrKey);
}

// ---------------------------------------------------------------------------
// Collide (+ stream/bin of the next step)
// ---------------------------------------------------------------------------
// Entry of next-step cell c in the window of the tile whose first cell is
// (x0, y0, z0): row r = (dz + 1) * 3 + (dy + 1) for the rows y0 + dy, z0 + dz
// (dy, dz in {-1, 0, 1}; periodic axes taken modulo L), column
// dx = (c_x - x0 + 1) mod L0 < WX = cells of the tile + 2.  False when the
// cell lies outside the window (the particle moved more than one cell).
template <bool W>
__device__ __forceinline__ bool win_entry(const int (&c)[3], int x0, int y0, int z0, int WX,
                                          int L0, int L1, int L2, int& r, int& dx) {
  dx = wrap1(c[0] - x0 + 1, L0);
  int dy = c[1] - y0;
  dy += L1 & -(int)(dy < -1);
  dy -= L1 & -(int)(dy > 1);
  int dz = c[2] - z0;
  if (!W) {
    dz += L2 & -(int)(dz < -1);
    dz -= L2 & -(int)(dz > 1);
  }
  r = (dz + 1) * 3 + (dy + 1);
  return (unsigned)dx < (unsigned)WX && (unsigned)(dy + 1) < 3u && (unsigned)(dz + 1) < 3u;
}

// Number of entries of seg[b..e) smaller than i (four independent LDS reads
// per trip so that they overlap).
__device__ __forceinline__ uint32_t rank_in_segment(const uint32_t* seg, uint32_t b, uint32_t e,
                                                    uint32_t i) {
  uint32_t r = 0, q = b;
  for (; q + 4 <= e; q += 4) {
    const uint32_t a0 = seg[q], a1 = seg[q + 1], a2 = seg[q + 2], a3 = seg[q + 3];
    r += (a0 < i ? 1u : 0u) + (a1 < i ? 1u : 0u) + (a2 < i ? 1u : 0u) + (a3 < i ? 1u : 0u);
  }
  for (; q < e; ++q) r += seg[q] < i ? 1u : 0u;
  return r;
}

// Per-cell record of the collision, FP64 forms: the update rotates with the
// vector formula in FP64.
struct CellLds {
  double V[3];   // centre-of-mass velocity
  double n[3];   // rotation axis
  double kappa;  // thermostat scale; 0 = the cell does not collide
};
// Split form: kappa R(alpha, n) built in FP64 and rounded to FP32, so the
// FP32 rotation's rounding differs from cell to cell (FP32 cos and sin of the
// one angle would bias every collision's energy the same way).
struct CellLdsSplit {
  float V[3];
  float R[9];    // kappa * rotation matrix, row major
  float coll;    // 0 = the cell does not collide
};
// SRD+a (Eqs. 3-4) adds the centre of mass in the cell frame and the angular
// velocity of the correction omega x r_ic.
struct CellLdsAmc : CellLds {
  double rc[3];
  double om[3];
};
struct CellLdsSplitAmc : CellLdsSplit {
  double rc[3];  // FP64: the correction is formed in FP64 and rounded once
  double om[3];
};
template <int F, bool A>
struct CellRec {
  using T = CellLds;
};
template <>
struct CellRec<kFormF64, true> {
  using T = CellLdsAmc;
};
template <>
struct CellRec<kFormF32, true> {
  using T = CellLdsAmc;
};
template <>
struct CellRec<kFormSplit, false> {
  using T = CellLdsSplit;
};
template <>
struct CellRec<kFormSplit, true> {
  using T = CellLdsSplitAmc;
};

// Position of a particle in the frame of its (shifted) cell, frac(x + s),
// from the stored coordinate (FP64 and FP32 forms: x; split form: the offset,
// whose cell index is an integer and drops out).  Exact for the FP32 forms.
template <typename X>
__device__ __forceinline__ double frame_pos(X x, double s) {
  const double y = (double)x + s;
  return y - floor(y);
}

// Rotation by alpha about n (Eq. 2): R u = cos(a) u + sin(a) n x u +
// (1 - cos(a)) (n . u) n.
template <typename T>
__device__ __forceinline__ void rotate(T ca, T sa, T omc, const T (&n)[3], const T (&u)[3],
                                       T (&r)[3]) {
  const T nu = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
  const T cx[3] = {n[1] * u[2] - n[2] * u[1], n[2] * u[0] - n[0] * u[2],
                   n[0] * u[1] - n[1] * u[0]};
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = ca * u[a] + sa * cx[a] + omc * nu * n[a];
}

// Sums of one cell by a pair of lanes (lane bit 0 = half): each lane sums
// half of the cell's fluid particles, sv[k][b..e) in canonical order (first
// half, then second), and the pair combines the halves in that order, so both
// lanes hold identical totals.  A wall-cut cell adds its phantoms' sums (ph,
// drawn by k_phantom_sums).  Every lane of the wavefront calls this (the pair
// exchanges values); only the first lane of a valid pair writes `out`.
__device__ __forceinline__ double pair_xor(double x) { return __shfl_xor(x, 1, 64); }
__device__ __forceinline__ float pair_xor(float x) { return __shfl_xor(x, 1, 64); }

// Fixed-point cell sums (Sec. III.C, reproducibility): a term x becomes the
// integer trunc(x 2^80) in 128-bit two's complement; sums are exact, hence
// independent of the order of the terms, and the value is the integer rounded
// once to FP64, times 2^-80.  Terms need |x| < 2^37 (no sum of at most 2^10
// terms can overflow); others (and NaN) set kErrFixRange.
struct Fix {
  uint64_t lo, hi;
};
__device__ __forceinline__ void fix_add(Fix& a, double x, uint32_t& err) {
  if (!(fabs(x) < 0x1p37)) {
    err |= kErrFixRange;
    return;
  }
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  const uint32_t ex = (uint32_t)(bits >> 52) & 0x7ffu;
  uint64_t mant = bits & 0x000fffffffffffffull;
  if (ex) mant |= 0x0010000000000000ull;
  // |x| 2^80 = mant 2^sh, sh = max(ex, 1) - 1075 + 80 <= 64 in range
  const int sh = (int)(ex ? ex : 1u) - 995;
  uint64_t lo, hi;
  if (sh >= 64) {
    lo = 0;
    hi = mant;
  } else if (sh > 0) {
    lo = mant << sh;
    hi = mant >> (64 - sh);
  } else {
    lo = -sh < 64 ? mant >> -sh : 0ull;  // truncation of the magnitude
    hi = 0;
  }
  if (bits >> 63) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  const uint64_t nlo = a.lo + lo;
  a.hi = a.hi + hi + (nlo < lo ? 1ull : 0ull);
  a.lo = nlo;
}
// Exact sum over the lane pair (both lanes hold the total).
__device__ __forceinline__ void fix_pair(Fix& a) {
  const uint64_t olo = (uint64_t)__shfl_xor((long long)a.lo, 1, 64);
  const uint64_t ohi = (uint64_t)__shfl_xor((long long)a.hi, 1, 64);
  const uint64_t nlo = a.lo + olo;
  a.hi = a.hi + ohi + (nlo < olo ? 1ull : 0ull);
  a.lo = nlo;
}
// Nearest FP64 of the integer, times 2^-80.  The 128-bit magnitude is
// normalised so that its top 64 bits carry the rounding position, with the
// bits below OR-ed into bit 0 (sticky); the u64 -> f64 conversion then rounds
// to nearest even once.
__device__ __forceinline__ double fix_value(Fix a) {
  const bool neg = (int64_t)a.hi < 0;
  uint64_t lo = a.lo, hi = a.hi;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  double d;
  if (hi == 0) {
    d = (double)lo * 0x1p-80;
  } else {
    const int lz = __clzll((long long)hi);
    const uint64_t top = lz ? (hi << lz) | (lo >> (64 - lz)) : hi;
    const uint64_t rest = lo << lz;
    d = ldexp((double)(top | (rest != 0ull ? 1ull : 0ull)), 64 - lz - 80);
  }
  return neg ? -d : d;
}

template <int F, bool W, bool M, bool A, bool X>
__device__ void cell_work(BoxRef B, uint32_t lkey, double sz, const CellDraw& cd,
                          const PhantomSums* __restrict__ ph,
                          const typename Form<F>::Vs* __restrict__ sv0,
                          const typename Form<F>::Vs* __restrict__ sv1,
                          const typename Form<F>::Vs* __restrict__ sv2,
                          const typename Form<F>::Xs* __restrict__ sx0,
                          const typename Form<F>::Xs* __restrict__ sx1,
                          const typename Form<F>::Xs* __restrict__ sx2, const double (&s)[3],
                          uint32_t b, uint32_t e, uint32_t half, bool valid,
                          typename CellRec<F, A>::T* out, uint32_t& err,
                          const int8_t* __restrict__ sside, double dle) {
  const uint32_t nf = valid ? e - b : 0u;
  const uint32_t mid = b + (nf + 1) / 2;
  const uint32_t qb = half ? mid : b, qe = valid ? (half ? e : mid) : b;
  uint32_t nph = 0;
  double pv[3] = {0.0, 0.0, 0.0}, pv2 = 0.0;
  if (W && !B.slip && valid && nf > 0) {
    const int cz = (int)(lkey / (uint32_t)(B.L[0] * B.L[1])) - 1;
    if (wall_fraction(sz, cz, B.L[2]) > 0.0) {
      nph = (uint32_t)ph->n;
      pv[0] = ph->v[0];
      pv[1] = ph->v[1];
      pv[2] = ph->v[2];
      pv2 = ph->v2;
    }
  }
  const uint32_t ntot = nf + nph;
  const double m = B.mass;
  double V[3];
  if constexpr (X) {
    // fixed-point momentum sums of the FP64 terms m v_i (every form)
    Fix fp[3] = {{0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}};
    for (uint32_t q = qb; q < qe; ++q) {
      fix_add(fp[0], m * (double)sv0[q], err);
      fix_add(fp[1], m * (double)sv1[q], err);
      fix_add(fp[2], m * (double)sv2[q], err);
    }
    double P[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fix_pair(fp[k]);
      P[k] = fix_value(fp[k]);
    }
    if (W && nph) {
#pragma unroll
      for (int k = 0; k < 3; ++k) P[k] = P[k] + m * pv[k];
    }
    const double Mtot = (double)(ntot ? ntot : 1u) * m;
    V[0] = P[0] / Mtot;
    V[1] = P[1] / Mtot;
    V[2] = P[2] / Mtot;
  } else if constexpr (F == kFormSplit) {
    // compensated FP32 momentum sums (Neumaier)
    const float mf = (float)m;
    float s[3] = {0.f, 0.f, 0.f}, c[3] = {0.f, 0.f, 0.f};
    auto add = [&](int k, float x) {
      const float tt = s[k] + x;
      if (fabsf(s[k]) >= fabsf(x)) {
        c[k] += (s[k] - tt) + x;
      } else {
        c[k] += (x - tt) + s[k];
      }
      s[k] = tt;
    };
#pragma unroll 4
    for (uint32_t q = qb; q < qe; ++q) {
      add(0, mf * sv0[q]);
      add(1, mf * sv1[q]);
      add(2, mf * sv2[q]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float os = pair_xor(s[k]), oc = pair_xor(c[k]);
      // first half's (s, c), then the second half's s added, then its c
      const float s0 = half ? os : s[k], c0 = half ? oc : c[k];
      const float s1 = half ? s[k] : os, c1 = half ? c[k] : oc;
      s[k] = s0;
      c[k] = c0;
      add(k, s1);
      c[k] += c1;
    }
    if (W && nph) {
#pragma unroll
      for (int k = 0; k < 3; ++k) add(k, (float)(m * pv[k]));
    }
    const float Mf = (float)(ntot ? ntot : 1u) * mf;
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k] = (double)((s[k] + c[k]) / Mf);
  } else {
    double P[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
    for (uint32_t q = qb; q < qe; ++q) {
      P[0] = P[0] + m * (double)sv0[q];
      P[1] = P[1] + m * (double)sv1[q];
      P[2] = P[2] + m * (double)sv2[q];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double o = pair_xor(P[k]);
      P[k] = half ? o + P[k] : P[k] + o;
    }
    if (W && nph) {
#pragma unroll
      for (int k = 0; k < 3; ++k) P[k] = P[k] + m * pv[k];
    }
    const double Mtot = (double)(ntot ? ntot : 1u) * m;
    V[0] = P[0] / Mtot;
    V[1] = P[1] / Mtot;
    V[2] = P[2] / Mtot;
  }
  double kappa = 1.0, K = 0.0;
  if (M) {
    if constexpr (X) {
      Fix fk = {0ull, 0ull};
      for (uint32_t q = qb; q < qe; ++q) {
        const double dx = (double)sv0[q] - V[0], dy = (double)sv1[q] - V[1],
                     dz = (double)sv2[q] - V[2];
        fix_add(fk, m * (dx * dx + dy * dy + dz * dz), err);
      }
      fix_pair(fk);
      K = fix_value(fk);
    } else {
#pragma unroll 4
      for (uint32_t q = qb; q < qe; ++q) {
        const double dx = (double)sv0[q] - V[0], dy = (double)sv1[q] - V[1],
                     dz = (double)sv2[q] - V[2];
        K = K + m * (dx * dx + dy * dy + dz * dz);
      }
      const double oK = pair_xor(K);
      K = half ? oK + K : K + oK;
    }
    if (W && nph) {
      // sum over phantoms of m |v - V|^2 from their velocity sums
      const double vV = pv[0] * V[0] + pv[1] * V[1] + pv[2] * V[2];
      const double VV = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
      K = K + m * (pv2 - 2.0 * vV + (double)nph * VV);
    }
    if (cd.Ek > 0.0 && K > 0.0) kappa = sqrt((2.0 * cd.Ek) / K);
  }
  // SRD+a (Eqs. 3-4, periodic boxes): omega = I^-1 dL with
  // dL = sum r_ic x (u_i - D u_i) and I the inertia tensor, both about the
  // centre of mass of the cell-frame positions (the mass m cancels; the
  // thermostat's energy below restores it).  A pair
  // uses the pseudo-inverse of its singular I (omega = dL / (tr I / 2), since
  // tr I = |r_1 - r_2|^2), three or more Cramer's rule, and det I = 0 gives
  // omega = 0.  Both lanes of the pair build identical totals.
  double rc[3] = {0.0, 0.0, 0.0}, om[3] = {0.0, 0.0, 0.0};
  if constexpr (A) {
    // cell-frame x; under Lees-Edwards shear a particle taken as its image
    // (sside = -1 / +1) sits at x - d / x + d
    auto fx = [&](uint32_t q) -> double {
      double xq = (double)sx0[q];
      if (sside) {
        if (sside[q] < 0) xq = xq - dle;
        if (sside[q] > 0) xq = xq + dle;
      }
      return frame_pos(xq, s[0]);
    };
    if constexpr (X) {
      Fix fr[3] = {{0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}};
      for (uint32_t q = qb; q < qe; ++q) {
        fix_add(fr[0], fx(q), err);
        fix_add(fr[1], frame_pos(sx1[q], s[1]), err);
        fix_add(fr[2], frame_pos(sx2[q], s[2]), err);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        fix_pair(fr[k]);
        rc[k] = fix_value(fr[k]) / (double)(nf ? nf : 1u);
      }
    } else {
      for (uint32_t q = qb; q < qe; ++q) {
        rc[0] = rc[0] + fx(q);
        rc[1] = rc[1] + frame_pos(sx1[q], s[1]);
        rc[2] = rc[2] + frame_pos(sx2[q], s[2]);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double o = pair_xor(rc[k]);
        rc[k] = (half ? o + rc[k] : rc[k] + o) / (double)(nf ? nf : 1u);
      }
    }
    // Moments about the centre of mass: M = sum r_ic u_i^T and S = sum r_ic
    // r_ic^T (15 sums, no per-particle rotation).  Then I = tr(S) 1 - S, the
    // angular momentum before the rotation L0 = eps : M, after it
    // L_D = sum r_ic x D u_i = eps : (M D^T), and dL = L0 - L_D.
    double mm[9], ss[6];  // mm[3a+b] = M_ab; ss: xx, yy, zz, xy, xz, yz
#pragma unroll
    for (int k = 0; k < 9; ++k) mm[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) ss[k] = 0.0;
    if constexpr (X) {
      // one pass per row a of M, with S_aa and S_a(a+1 mod 3): five exact
      // sums live at a time
#pragma unroll 1
      for (int a = 0; a < 3; ++a) {
        Fix f5[5] = {{0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}};
        const int a1 = a == 2 ? 0 : a + 1;
        for (uint32_t q = qb; q < qe; ++q) {
          const double r[3] = {fx(q) - rc[0], frame_pos(sx1[q], s[1]) - rc[1],
                               frame_pos(sx2[q], s[2]) - rc[2]};
          const double u[3] = {(double)sv0[q] - V[0], (double)sv1[q] - V[1],
                               (double)sv2[q] - V[2]};
          const double ra = a == 0 ? r[0] : (a == 1 ? r[1] : r[2]);
          const double rb = a1 == 0 ? r[0] : (a1 == 1 ? r[1] : r[2]);
          fix_add(f5[0], ra * u[0], err);
          fix_add(f5[1], ra * u[1], err);
          fix_add(f5[2], ra * u[2], err);
          fix_add(f5[3], ra * ra, err);
          fix_add(f5[4], ra * rb, err);
        }
        double v5[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          fix_pair(f5[k]);
          v5[k] = fix_value(f5[k]);
        }
        // scatter into mm / ss (ss: xx, yy, zz, xy, xz, yz; a = 2 gives zx = xz)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2) {
          if (a == 0) mm[b2] = v5[b2];
          if (a == 1) mm[3 + b2] = v5[b2];
          if (a == 2) mm[6 + b2] = v5[b2];
        }
        if (a == 0) { ss[0] = v5[3]; ss[3] = v5[4]; }
        if (a == 1) { ss[1] = v5[3]; ss[5] = v5[4]; }
        if (a == 2) { ss[2] = v5[3]; ss[4] = v5[4]; }
      }
    } else {
    for (uint32_t q = qb; q < qe; ++q) {
      const double r[3] = {fx(q) - rc[0], frame_pos(sx1[q], s[1]) - rc[1],
                           frame_pos(sx2[q], s[2]) - rc[2]};
      const double u[3] = {(double)sv0[q] - V[0], (double)sv1[q] - V[1], (double)sv2[q] - V[2]};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2) mm[3 * a + b2] = fma(r[a], u[b2], mm[3 * a + b2]);
      ss[0] = fma(r[0], r[0], ss[0]);
      ss[1] = fma(r[1], r[1], ss[1]);
      ss[2] = fma(r[2], r[2], ss[2]);
      ss[3] = fma(r[0], r[1], ss[3]);
      ss[4] = fma(r[0], r[2], ss[4]);
      ss[5] = fma(r[1], r[2], ss[5]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double o = pair_xor(mm[k]);
      mm[k] = half ? o + mm[k] : mm[k] + o;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double o = pair_xor(ss[k]);
      ss[k] = half ? o + ss[k] : ss[k] + o;
    }
    }
    const double xx = ss[1] + ss[2], yy = ss[0] + ss[2], zz = ss[0] + ss[1];
    const double xy = -ss[3], xz = -ss[4], yz = -ss[5];
    // rotation matrix D(alpha, n), row major
    const double n[3] = {cd.n[0], cd.n[1], cd.n[2]};
    const double ca = B.ca, sa = B.sa, omc = B.omc;
    const double D[9] = {ca + omc * n[0] * n[0],        omc * n[0] * n[1] - sa * n[2],
                         omc * n[0] * n[2] + sa * n[1], omc * n[1] * n[0] + sa * n[2],
                         ca + omc * n[1] * n[1],        omc * n[1] * n[2] - sa * n[0],
                         omc * n[2] * n[0] - sa * n[1], omc * n[2] * n[1] + sa * n[0],
                         ca + omc * n[2] * n[2]};
    // (M D^T)_bc = row b of M . row c of D
    auto md = [&](int b2, int c) {
      return mm[3 * b2] * D[3 * c] + mm[3 * b2 + 1] * D[3 * c + 1] + mm[3 * b2 + 2] * D[3 * c + 2];
    };
    const double LD[3] = {md(1, 2) - md(2, 1), md(2, 0) - md(0, 2), md(0, 1) - md(1, 0)};
    double a9[3] = {(mm[5] - mm[7]) - LD[0], (mm[6] - mm[2]) - LD[1], (mm[1] - mm[3]) - LD[2]};
    if (nf == 2) {
      const double hm = 0.5 * (xx + yy + zz);
      if (hm > 0.0) {
        const double ih = 1.0 / hm;
#pragma unroll
        for (int k = 0; k < 3; ++k) om[k] = a9[k] * ih;
      }
    } else if (nf >= 3) {
      // adjugate of the symmetric I
      const double c00 = yy * zz - yz * yz, c01 = xz * yz - xy * zz, c02 = xy * yz - yy * xz;
      const double c11 = xx * zz - xz * xz, c12 = xy * xz - xx * yz, c22 = xx * yy - xy * xy;
      const double det = xx * c00 + xy * c01 + xz * c02;
      if (det != 0.0) {
        const double id = 1.0 / det;
        om[0] = (c00 * a9[0] + c01 * a9[1] + c02 * a9[2]) * id;
        om[1] = (c01 * a9[0] + c11 * a9[1] + c12 * a9[2]) * id;
        om[2] = (c02 * a9[0] + c12 * a9[1] + c22 * a9[2]) * id;
      }
    }
    if constexpr (M) {
      // the thermostat scales the corrected relative velocities D u_i +
      // omega x r_ic to the drawn energy; their kinetic energy is
      // K + m (2 omega . L_D + omega . I omega), K that of the u_i
      kappa = 1.0;
      if (cd.Ek > 0.0) {
        const double Io[3] = {xx * om[0] + xy * om[1] + xz * om[2],
                              xy * om[0] + yy * om[1] + yz * om[2],
                              xz * om[0] + yz * om[1] + zz * om[2]};
        double cr = 0.0, q = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          cr = cr + om[k] * LD[k];
          q = q + om[k] * Io[k];
        }
        const double K2 = K + m * (2.0 * cr + q);
        if (K2 > 0.0) kappa = sqrt((2.0 * cd.Ek) / K2);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) om[k] = kappa * om[k];
    }
  }
  if (!valid || half) return;
  // cells that do not collide keep v exactly (kappa = 0 / coll = 0 marks them)
  const bool coll = nf > 0 && ntot >= 2;
  if constexpr (A) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      out->rc[k] = rc[k];
      out->om[k] = coll ? om[k] : 0.0;
    }
  }
  if constexpr (F == kFormSplit) {
    const double n[3] = {cd.n[0], cd.n[1], cd.n[2]};
    const double ca = B.ca, sa = B.sa, omc = B.omc;
    const double R[9] = {ca + omc * n[0] * n[0],        omc * n[0] * n[1] - sa * n[2],
                         omc * n[0] * n[2] + sa * n[1], omc * n[1] * n[0] + sa * n[2],
                         ca + omc * n[1] * n[1],        omc * n[1] * n[2] - sa * n[0],
                         omc * n[2] * n[0] - sa * n[1], omc * n[2] * n[1] + sa * n[0],
                         ca + omc * n[2] * n[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k) out->V[k] = coll ? (float)V[k] : 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) out->R[k] = coll ? (float)(kappa * R[k]) : 0.0f;
    out->coll = coll ? 1.0f : 0.0f;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      out->V[k] = coll ? V[k] : 0.0;
      out->n[k] = coll ? cd.n[k] : 0.0;
    }
    out->kappa = coll ? kappa : 0.0;
  }
}

// The collide workgroup is a single wavefront.  LDS instructions of one wave
// execute in issue order, so lanes see each other's LDS writes without a
// hardware barrier; a wavefront-scope fence keeps the compiler from moving LDS
// accesses across phase boundaries.  (A workgroup barrier would also wait for
// every outstanding global load and store of the wave.)
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Tile index of the it-th work item of this workgroup (XCD-aware order:
// workgroup b runs on XCD b % 8; each XCD takes a contiguous part of the tile
// list, which the host ordered so that neighbouring rows are close in it).
struct TileWalk {
  uint32_t first, stride, per_xcd, xcd, ntiles;
  __device__ uint32_t tile(uint32_t it) const {
    if (per_xcd) {
      if (it >= per_xcd) return 0xffffffffu;
      const uint32_t t = xcd * per_xcd + it;
      return t < ntiles ? t : 0xffffffffu;
    }
    return it < ntiles ? it : 0xffffffffu;
  }
};

template <int F, bool W, bool M, bool A, bool X, bool E>
__global__ __launch_bounds__(kCollideThreads) __attribute__((amdgpu_waves_per_eu((W || A || X) ? 2 : 3)))
void k_collide(Dev d, uint32_t ntiles, int xcd_remap) {
  using Fm = Form<F>;
  using Vs = typename Fm::Vs;
  using Xs = typename Fm::Xs;
  constexpr int NT = kCollideThreads;
  constexpr int NS = kTileCap / kCollideThreads;
  static_assert(kTileMaxCells < NT, "one lane per cell offset (nc + 1) of a tile");
  static_assert(2 * kTileMaxCells <= NT, "two lanes per cell in the cell sums");
  static_assert(NT == 64, "the workgroup is one wavefront (see wave_sync)");
  __shared__ uint32_t s_off[kTileMaxCells + 1];
  __shared__ uint32_t s_idx[kTileCap];   // perm entries, segment order as scattered
  __shared__ uint32_t s_rk[kTileCap];    // logical index of each entry (ids tracked)
  __shared__ uint32_t s_idc[kTileCap];   // logical index at the canonical position
  __shared__ uint8_t s_lc[kTileCap];     // local cell of each slot
  __shared__ Vs s_v[3][kTileCap];        // streamed velocities, canonical order
  __shared__ Xs s_x[3][kTileCap];        // streamed positions (offsets), canonical order
  __shared__ uint32_t s_c[Fm::kHasCell ? kTileCap : 1];
  __shared__ typename CellRec<F, A>::T s_cell[kTileMaxCells];
  __shared__ int8_t s_side[E ? kTileCap : 1];  // Lees-Edwards side of each slot
  __shared__ double s_sh[8];  // shifts of t and t + 1; Lees-Edwards offsets of t + 1, t + 2
  // next-step window of the tile: cells x0-1 .. x0+nc of the rows (y0 +- 1,
  // z0 +- 1), plus one entry for particles that leave it; per pass: counts,
  // then their exclusive prefix (the output order of the pass)
  constexpr int kWin = 9 * (kTileMaxCells + 2) + 1;
  __shared__ uint32_t s_pc[kWin];

  const uint64_t t = as_const(d.ctrl)->step;
  const uint32_t cur = as_const(d.ctrl)->cur;
  const int32_t R = as_const(d.ctrl)->reorder;
  // the state is always written into the other buffer (cell by cell, each
  // tile pass grouped by next-step cell); logical indices are renumbered to
  // the canonical (cell, index) order on reorder steps
  const bool renumber = R > 0 && (t + 1) % (uint64_t)R == 0;
  const StatePtrs in = d.S[cur];
  const StatePtrs out = d.S[cur ^ 1u];
  uint32_t err = 0;
  const uint32_t lane = threadIdx.x;

  TileWalk walk;
  walk.ntiles = ntiles;
  walk.first = blockIdx.x;
  walk.stride = gridDim.x;
  walk.per_xcd = 0;
  walk.xcd = 0;
  if (xcd_remap && gridDim.x % 8 == 0) {
    walk.xcd = blockIdx.x % 8;
    walk.per_xcd = (ntiles + 7) / 8;
    walk.first = blockIdx.x / 8;
    walk.stride = gridDim.x / 8;
  }

  // Software pipeline over tiles: offsets are fetched two tiles ahead, the
  // first pass's perm entries and the cell draws one tile ahead.
  uint32_t it = walk.first;
  uint32_t tcur = walk.tile(it);
  uint32_t tnext = walk.tile(it + walk.stride);
  uint32_t off_cur = 0, off_next = 0;
  if (tcur != 0xffffffffu) {
    const Tile Tc = load_tile(d.tiles, tcur);
    if (lane <= Tc.nc) off_cur = d.offset[Tc.c0 + lane];
  }
  if (tnext != 0xffffffffu) {
    const Tile Tn = load_tile(d.tiles, tnext);
    if (lane <= Tn.nc) off_next = d.offset[Tn.c0 + lane];
  }
  uint32_t perm_cur[NS];
  CellDraw draw_cur;
  bool have_pf = false;  // perm_cur / draw_cur hold the current tile's data
  uint32_t cached_box = 0xffffffffu;

  for (; tcur != 0xffffffffu; it += walk.stride) {
    const Tile T = load_tile(d.tiles, tcur);
    BoxRef B = as_const(d.boxes)[T.box];
    const uint32_t tafter = walk.tile(it + 2 * walk.stride);
    wave_sync();  // LDS of the previous tile is free
    if (lane <= T.nc) s_off[lane] = off_cur;
    if (lane == 0 && T.box != cached_box) {
      double s0[3], s1[3];
      shift_of(B, t, s0);
      shift_of(B, t + 1, s1);
      s_sh[0] = s0[0];
      s_sh[1] = s0[1];
      s_sh[2] = s0[2];
      s_sh[3] = s1[0];
      s_sh[4] = s1[1];
      s_sh[5] = s1[2];
      s_sh[6] = E ? le_offset(B, t + 1) : 0.0;
      s_sh[7] = E ? le_offset(B, t + 2) : 0.0;
    }
    cached_box = T.box;
    const uint32_t lkey0 = T.c0 - B.cbase;
    // tiles lie inside one row: (x0 .. x0 + nc - 1, y0, z0)
    const int x0 = (int)T.x0, y0 = (int)T.y0, z0 = (int)T.z0;
    const int WX = (int)T.nc + 2;
    const int L0 = B.L[0], L1 = B.L[1], L2 = B.L[2];
    // offsets of the tile after next (two ahead)
    uint32_t off_after = 0;
    if (tafter != 0xffffffffu) {
      const Tile Ta = load_tile(d.tiles, tafter);
      if (lane <= Ta.nc) off_after = d.offset[Ta.c0 + lane];
    }
    wave_sync();

    uint32_t perm_next[NS];
    CellDraw draw_next;
    bool issued_next = false;

    uint32_t cs = 0;
    while (cs < T.nc) {
      const uint32_t base = s_off[cs];
      // largest ce in (cs, nc] with s_off[ce] - base <= capacity
      uint32_t ce;
      if (s_off[T.nc] - base <= (uint32_t)kTileCap) {
        ce = T.nc;
      } else {
        uint32_t lo = cs + 1, hi = T.nc;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (s_off[mid] - base <= (uint32_t)kTileCap) {
            lo = mid;
          } else {
            hi = mid;
          }
        }
        ce = lo;
      }
      if (s_off[ce] < base || s_off[ce] > d.ntot) {  // inconsistent offsets: stop
        err |= kErrKey;
        break;
      }
      const uint32_t np = s_off[ce] - base;
      const bool use_pf = have_pf && cs == 0;

      if (np > (uint32_t)kTileCap) {
        // one cell beyond capacity: stream and re-bin its particles unchanged
        err |= kErrCellOverflow;
        const double snx[3] = {s_sh[3], s_sh[4], s_sh[5]};
        for (uint32_t q0 = 0; q0 < np; q0 += NT) {
          const uint32_t q = q0 + lane;
          const uint32_t i = q < np ? d.perm[base + q] : d.ntot;
          const bool live = i < d.ntot;
          uint32_t kn = 0;
          if (live) {
            typename Fm::P p;
            typename Fm::Vv v;
            uint32_t id;
            Fm::load_all(in, i, p, v, id);
            Fm::template stream<W>(p, v, B, s_sh[6], E && B.le);
            const uint32_t j = base + q;
            Fm::store_all(out, j, p, v, renumber ? j : id);
            Fm::template stream<W>(p, v, B, s_sh[7], E && B.le);
            kn = B.cbase + Fm::template key<W>(p, snx, B, err, s_sh[7], E && B.le);
            d.key[j] = kn;
          }
          const uint32_t rk = wave_hist_rank(d.hist, kn, live);
          if (live) d.rank[base + q] = (uint16_t)min(rk, 0xffffu);
        }
        cs = ce;
        wave_sync();
        continue;
      }

      // Phase A: segment entries (prefetched for the first pass) and their
      // cell
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t q = lane + k * NT;
        if (q < np) s_idx[q] = use_pf ? perm_cur[k] : d.perm[base + q];
      }
      if (cs + lane < ce) {
        const uint32_t c = cs + lane;
        const uint32_t b = s_off[c] - base, e = s_off[c + 1] - base;
        for (uint32_t q = b; q < e; ++q) s_lc[q] = (uint8_t)(c - cs);
      }
      wave_sync();

      // Phase B: gather, canonical position (rank by logical index inside
      // the cell), stream of step t, park in LDS.
      {
        // the logical indices are gathered with the state (one memory round
        // trip per pass), then put in LDS for the in-cell ranking
        typename Fm::P p[NS];
        typename Fm::Vv v[NS];
        uint32_t ii[NS], idk[NS];
        // issue the gathers ahead of other waves' arithmetic
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const uint32_t q = lane + k * NT;
          ii[k] = 0;
          idk[k] = 0;
          if (q < np) {
            ii[k] = s_idx[q] < d.ntot ? s_idx[q] : 0u;
            Fm::load_all(in, ii[k], p[k], v[k], idk[k]);
          }
        }
        // prefetch the next tile's first-pass perm entries and cell draws
        if (!issued_next && tnext != 0xffffffffu) {
          issued_next = true;
          const Tile Tn = load_tile(d.tiles, tnext);
          const uint32_t nb = (uint32_t)__builtin_amdgcn_readfirstlane((int)off_next);
          const uint32_t ne = (uint32_t)__builtin_amdgcn_readlane((int)off_next, Tn.nc);
          const uint32_t nn = ne >= nb ? ne - nb : 0u;
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            const uint32_t q = lane + k * NT;
            perm_next[k] = (q < nn && nb + q < d.ntot) ? d.perm[nb + q] : 0u;
          }
          if (lane < Tn.nc) draw_next = d.draws[Tn.c0 + lane];
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const uint32_t q = lane + k * NT;
          if (q < np) s_rk[q] = idk[k];
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const uint32_t q = lane + k * NT;
          __builtin_amdgcn_sched_barrier(0);
          if (q < np) {
            const uint32_t c = cs + s_lc[q];
            const uint32_t b = s_off[c] - base, e = s_off[c + 1] - base;
            const uint32_t id = s_rk[q];
            const uint32_t qc = b + rank_in_segment(s_rk, b, e, id);
            Fm::template stream<W>(p[k], v[k], B, s_sh[6], E && B.le);
            if constexpr (E) {
              const int side = B.le ? Fm::le_side(p[k], s_sh[2], B) : 0;
              s_side[qc] = (int8_t)side;
              if (e - b >= 2u) {
                // a colliding cell across a z face: its image's velocity frame
                if (side < 0) v[k].v[0] = (Vs)((double)v[k].v[0] - B.leu);
                if (side > 0) v[k].v[0] = (Vs)((double)v[k].v[0] + B.leu);
              }
            }
            Fm::to_lds(p[k], s_x[0], s_x[1], s_x[2], s_c, qc);
            s_v[0][qc] = v[k].v[0];
            s_v[1][qc] = v[k].v[1];
            s_v[2][qc] = v[k].v[2];
            s_idc[qc] = id;
          }
        }
      }
      wave_sync();

      // Phase C: two lanes per cell (lanes 2j and 2j + 1 for cell cs + j); the
      // first pass uses the prefetched draws, which lane j holds
      {
        const uint32_t j = lane >> 1;
        const uint32_t c = cs + j;
        const bool valid = c < ce;
        const uint32_t b = valid ? s_off[c] - base : 0u, e = valid ? s_off[c + 1] - base : 0u;
        CellDraw cd;
#pragma unroll
        for (int k = 0; k < 3; ++k) cd.n[k] = __shfl(draw_cur.n[k], (int)j, 64);
        cd.Ek = __shfl(draw_cur.Ek, (int)j, 64);
        if (!use_pf) {
          if (valid && e > b) {
            cd = d.draws[T.c0 + c];
          } else {
            cd.n[0] = cd.n[1] = cd.n[2] = 0.0;
            cd.Ek = 0.0;
          }
        }
        const double s_t[3] = {s_sh[0], s_sh[1], s_sh[2]};
        cell_work<F, W, M, A, X>(B, lkey0 + c, s_sh[2], cd,
                                 W ? d.phs + T.c0 + (valid ? c : 0u) : nullptr, s_v[0], s_v[1],
                                 s_v[2], s_x[0], s_x[1], s_x[2], s_t, b, e, lane & 1u, valid,
                                 &s_cell[j], err, E ? s_side : nullptr, s_sh[6]);
      }
      wave_sync();

      // Phase D1: rotate + scale, gravity; the next step's cell of each
      // particle and its rank among the pass's particles going there
      for (int i = (int)lane; i < 9 * WX + 1; i += NT) s_pc[i] = 0u;
      wave_sync();
      const double snext[3] = {s_sh[3], s_sh[4], s_sh[5]};
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t q = lane + k * NT;
        __builtin_amdgcn_sched_barrier(0);
        if (q < np) {
          typename Fm::P p;
          typename Fm::Vv v;
          Fm::from_lds(p, s_x[0], s_x[1], s_x[2], s_c, q);
          v.v[0] = s_v[0][q];
          v.v[1] = s_v[1][q];
          v.v[2] = s_v[2][q];
          const auto& C = s_cell[s_lc[q]];
          if constexpr (F == kFormSplit) {
            if (C.coll != 0.0f) {
              const float u[3] = {v.v[0] - C.V[0], v.v[1] - C.V[1], v.v[2] - C.V[2]};
#pragma unroll
              for (int a = 0; a < 3; ++a)
                v.v[a] = C.V[a] + fmaf(C.R[3 * a], u[0], fmaf(C.R[3 * a + 1], u[1], C.R[3 * a + 2] * u[2]));
              if constexpr (A) {
                // omega x r_ic in FP64 (|omega| is large in ill-conditioned
                // cells), added to the FP32 rotation result with one rounding
                double xq = (double)s_x[0][q];
                if constexpr (E) {
                  if (s_side[q] < 0) xq = xq - s_sh[6];
                  if (s_side[q] > 0) xq = xq + s_sh[6];
                }
                const double r[3] = {frame_pos(xq, s_sh[0]) - C.rc[0],
                                     frame_pos(s_x[1][q], s_sh[1]) - C.rc[1],
                                     frame_pos(s_x[2][q], s_sh[2]) - C.rc[2]};
                v.v[0] = (float)((double)v.v[0] + (C.om[1] * r[2] - C.om[2] * r[1]));
                v.v[1] = (float)((double)v.v[1] + (C.om[2] * r[0] - C.om[0] * r[2]));
                v.v[2] = (float)((double)v.v[2] + (C.om[0] * r[1] - C.om[1] * r[0]));
              }
              if constexpr (E) {  // leave the Lees-Edwards image frame
                if (s_side[q] < 0) v.v[0] = (float)((double)v.v[0] + B.leu);
                if (s_side[q] > 0) v.v[0] = (float)((double)v.v[0] - B.leu);
              }
            }
            if (B.grav) {
#pragma unroll
              for (int a = 0; a < 3; ++a) v.v[a] = v.v[a] + (float)B.gh[a];
            }
          } else {
            double w[3] = {(double)v.v[0], (double)v.v[1], (double)v.v[2]};
            if (C.kappa != 0.0) {
              const double u[3] = {w[0] - C.V[0], w[1] - C.V[1], w[2] - C.V[2]};
              const double nd[3] = {C.n[0], C.n[1], C.n[2]};
              double r[3];
              rotate<double>(B.ca, B.sa, B.omc, nd, u, r);
#pragma unroll
              for (int a = 0; a < 3; ++a) w[a] = C.V[a] + C.kappa * r[a];
              if constexpr (A) {
                double xq = (double)s_x[0][q];
                if constexpr (E) {
                  if (s_side[q] < 0) xq = xq - s_sh[6];
                  if (s_side[q] > 0) xq = xq + s_sh[6];
                }
                const double rr[3] = {frame_pos(xq, s_sh[0]) - C.rc[0],
                                      frame_pos(s_x[1][q], s_sh[1]) - C.rc[1],
                                      frame_pos(s_x[2][q], s_sh[2]) - C.rc[2]};
                w[0] = w[0] + (C.om[1] * rr[2] - C.om[2] * rr[1]);
                w[1] = w[1] + (C.om[2] * rr[0] - C.om[0] * rr[2]);
                w[2] = w[2] + (C.om[0] * rr[1] - C.om[1] * rr[0]);
              }
              if constexpr (E) {  // leave the Lees-Edwards image frame
                if (s_side[q] < 0) w[0] = w[0] + B.leu;
                if (s_side[q] > 0) w[0] = w[0] - B.leu;
              }
            }
            if (B.grav) {
#pragma unroll
              for (int a = 0; a < 3; ++a) w[a] = w[a] + B.gh[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) v.v[a] = (Vs)w[a];
          }
          // v' back in place; the next step's cell and its window entry
          s_v[0][q] = v.v[0];
          s_v[1][q] = v.v[1];
          s_v[2][q] = v.v[2];
          Fm::template stream<W>(p, v, B, s_sh[7], E && B.le);
          int c[3];
          Fm::template coords<W>(p, snext, B, c, err, s_sh[7], E && B.le);
          const uint32_t kn = B.cbase + linear_key(c, B);
          int r, dx;
          uint32_t e = (uint32_t)(9 * WX);  // outside the window: counted in D2
          if (win_entry<W>(c, x0, y0, z0, WX, L0, L1, L2, r, dx)) e = (uint32_t)(r * WX + dx);
          const uint32_t rank = atomicAdd(&s_pc[e], 1u);
          s_idx[q] = e << 16 | rank;
          s_rk[q] = kn;
        }
      }
      wave_sync();
      // Per window entry (5 per lane): add the pass's count to the next
      // step's histogram, whose old value is the rank base of these particles
      // in their cell (used after D2, so that the atomics' latency overlaps
      // the stores); and the exclusive prefix of the counts, which orders the
      // pass's output.
      uint32_t rb5[5];
      {
        const int ne = 9 * WX + 1;
        const int i0 = (int)lane * 5;
        uint32_t cnt5[5];
        uint32_t sum = 0;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const int i = i0 + m;
          cnt5[m] = i < ne ? s_pc[i] : 0u;
          sum += cnt5[m];
          rb5[m] = 0u;
          if (i < ne - 1 && cnt5[m]) {
            const int rr = i / WX, dx = i - rr * WX;
            int c[3] = {x0 - 1 + dx, y0 + rr % 3 - 1, z0 + rr / 3 - 1};
            c[0] = wrap1(c[0], L0);
            c[1] = wrap1(c[1], L1);
            if (!W) c[2] = wrap1(c[2], L2);
            rb5[m] = atomicAdd(&d.hist[B.cbase + linear_key(c, B)], cnt5[m]);
          }
        }
        const uint32_t incl = wave_inclusive_scan(sum);
        uint32_t run = incl - sum;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          if (i0 + m < ne) s_pc[i0 + m] = run;
          run += cnt5[m];
        }
      }
      wave_sync();
      // D2: the pass's particles, grouped by next-step cell, into its slots;
      // logical indices: the canonical (cell, index) position on reorder steps
      __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t q = lane + k * NT;
        __builtin_amdgcn_sched_barrier(0);
        if (q < np) {
          const uint32_t pk = s_idx[q];
          const uint32_t j = base + s_pc[pk >> 16] + (pk & 0xffffu);
          const uint32_t kn = s_rk[q];
          s_rk[q] = j;
          if (j < d.ntot && j < base + np) {
            typename Fm::P p;
            typename Fm::Vv v;
            Fm::from_lds(p, s_x[0], s_x[1], s_x[2], s_c, q);
            v.v[0] = s_v[0][q];
            v.v[1] = s_v[1][q];
            v.v[2] = s_v[2][q];
            Fm::store_all(out, j, p, v, renumber ? base + q : s_idc[q]);
            d.key[j] = kn;
            // leaving the window: counted one by one
            if ((pk >> 16) == (uint32_t)(9 * WX))
              d.rank[j] = (uint16_t)min(atomicAdd(&d.hist[kn], 1u), 0xffffu);
          } else {
            err |= kErrKey;
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
      // D3: ranks inside the next-step cells (rank base of the entry + place)
      wave_sync();
      {
        const int ne = 9 * WX + 1;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const int i = (int)lane * 5 + m;
          if (rb5[m] > 0xffffu) {
            err |= kErrCellOverflow;
            rb5[m] = 0xffffu;
          }
          if (i < ne) s_pc[i] = rb5[m];
        }
      }
      wave_sync();
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t q = lane + k * NT;
        if (q < np) {
          const uint32_t pk = s_idx[q];
          const uint32_t j = s_rk[q];
          if ((pk >> 16) != (uint32_t)(9 * WX) && j < d.ntot && j < base + np)
            d.rank[j] = (uint16_t)min(s_pc[pk >> 16] + (pk & 0xffffu), 0xffffu);
        }
      }
      cs = ce;
      wave_sync();
    }
    // advance the pipeline
    tcur = tnext;
    tnext = tafter;
    off_cur = off_next;
    off_next = off_after;
    have_pf = issued_next;
    if (issued_next) {
#pragma unroll
      for (int k = 0; k < NS; ++k) perm_cur[k] = perm_next[k];
      draw_cur = draw_next;
    }
  }
  if (err) atomicOr(&d.ctrl->err, err);
}

// Runtime flags (form, walls, thermostat, SRD+a, fixed-point sums,
// Lees-Edwards) -> the k_collide instantiation.  SRD+a next to walls runs
// with slip walls only (the host refuses it with no-slip walls).
struct CollideLaunchOp {
  template <int F, bool W, bool M, bool A, bool X, bool E>
  static hipError_t run(const Dev& d, const Launch& l, int*) {
    hipLaunchKernelGGL((k_collide<F, W, M, A, X, E>), dim3(l.collide_grid),
                       dim3(kCollideThreads), 0, l.stream, d, (uint32_t)l.ntiles, l.xcd_remap);
    return hipGetLastError();
  }
};
struct CollideOccOp {
  template <int F, bool W, bool M, bool A, bool X, bool E>
  static hipError_t run(const Dev&, const Launch&, int* n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_collide<F, W, M, A, X, E>,
                                                        kCollideThreads, 0);
  }
};
// Lees-Edwards (E) is built for periodic boxes only.
template <class Op, int F, bool W, bool M, bool A, bool X>
static hipError_t collide_pick_e(const Dev& d, const Launch& l, int* n) {
  if constexpr (W) {
    return l.le ? hipErrorInvalidValue : Op::template run<F, W, M, A, X, false>(d, l, n);
  } else {
    return l.le ? Op::template run<F, W, M, A, X, true>(d, l, n)
                : Op::template run<F, W, M, A, X, false>(d, l, n);
  }
}
template <class Op, int F, bool W, bool M, bool A>
static hipError_t collide_pick_x(const Dev& d, const Launch& l, int* n) {
  return l.fixed ? collide_pick_e<Op, F, W, M, A, true>(d, l, n)
                 : collide_pick_e<Op, F, W, M, A, false>(d, l, n);
}
template <class Op, int F, bool W, bool M>
static hipError_t collide_pick_a(const Dev& d, const Launch& l, int* n) {
  return l.amc ? collide_pick_x<Op, F, W, M, true>(d, l, n)
               : collide_pick_x<Op, F, W, M, false>(d, l, n);
}
template <class Op, int F, bool W>
static hipError_t collide_pick_m(const Dev& d, const Launch& l, int* n) {
  return l.mbs ? collide_pick_a<Op, F, W, true>(d, l, n) : collide_pick_a<Op, F, W, false>(d, l, n);
}
template <class Op, int F>
static hipError_t collide_pick_w(const Dev& d, const Launch& l, int* n) {
  return l.walls ? collide_pick_m<Op, F, true>(d, l, n) : collide_pick_m<Op, F, false>(d, l, n);
}
template <class Op>
static hipError_t collide_dispatch(const Dev& d, const Launch& l, int* n) {
  switch (l.form) {
    case kFormF64: return collide_pick_w<Op, kFormF64>(d, l, n);
    case kFormF32: return collide_pick_w<Op, kFormF32>(d, l, n);
    case kFormSplit: return collide_pick_w<Op, kFormSplit>(d, l, n);
    default: return hipErrorInvalidValue;
  }
}

hipError_t collide_occupancy(const Launch& l, int* blocks_per_cu) {
  return collide_dispatch<CollideOccOp>(Dev{}, l, blocks_per_cu);
}

// ---------------------------------------------------------------------------
// Canonical permutation for export: sort each cell segment by logical index
// (ids[slot * stride], or the slot itself when ids is null).
// ---------------------------------------------------------------------------
__global__ void k_canon_perm(uint32_t* __restrict__ perm, const uint32_t* __restrict__ offset,
                             uint64_t ncell, uint32_t n, const uint32_t* __restrict__ ids,
                             uint32_t stride) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const uint32_t b = offset[c], e = offset[c + 1];
  if (e > n || b > e) return;
  auto rk = [&](uint32_t slot) { return ids && slot < n ? ids[(size_t)slot * stride] : slot; };
  for (uint32_t i = b + 1; i < e; ++i) {
    const uint32_t x = perm[i];
    const uint32_t kx = rk(x);
    uint32_t j = i;
    while (j > b && rk(perm[j - 1]) > kx) {
      perm[j] = perm[j - 1];
      --j;
    }
    perm[j] = x;
  }
}

// ---------------------------------------------------------------------------
// Sampled state: the inverse of one box's logical-index array, then a gather
// of selected logical particles as FP64 in cell units (the split form's
// cell + offset is exact in FP64).  A logical index with no stored slot
// yields NaN.
// ---------------------------------------------------------------------------
__global__ void k_invert_ids(const uint32_t* __restrict__ id, uint32_t id_stride, uint32_t pbase,
                             uint32_t np, uint32_t* __restrict__ inv) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < np; q += stride) {
    const uint32_t j = pbase + (uint32_t)q;
    const uint32_t l = id[(size_t)j * id_stride] - pbase;
    if (l < np) inv[l] = j;
  }
}

template <int F>
__global__ __launch_bounds__(kThreads) void k_gather_particles(StatePtrs S,
                                                                const uint32_t* __restrict__ inv,
                                                                uint32_t pbase, uint32_t np,
                                                                const uint32_t* __restrict__ lidx,
                                                                uint32_t m, double* __restrict__ out) {
  const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= m) return;
  const uint32_t l = lidx[k];
  uint32_t j = 0xffffffffu;
  if (l < np) j = inv ? inv[l] : pbase + l;
  double r[6];
  if (j == 0xffffffffu || j - pbase >= np) {
#pragma unroll
    for (int c = 0; c < 6; ++c) r[c] = __builtin_nan("");
  } else if constexpr (F == kFormF64) {
    const RecF64 q = ((const RecF64*)S.rec)[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = q.x[c];
      r[3 + c] = q.v[c];
    }
  } else if constexpr (F == kFormF32) {
    const RecF32 q = ((const RecF32*)S.rec)[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = (double)q.x[c];
      r[3 + c] = (double)q.v[c];
    }
  } else {
    const RecSplit q = ((const RecSplit*)S.rec)[j];
    int ci[3];
    split_decode(q.cell, ci);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = (double)ci[c] + (double)q.o[c];
      r[3 + c] = (double)q.v[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) out[(uint64_t)c * m + k] = r[c];
}

// ---------------------------------------------------------------------------
// FP64 state of box 0 from / to caller-owned device arrays x[3][n], v[3][n]
// in physical units (the allocation-free entry point).  Load: cell units
// (x / a, v / a) into state buffer `cur`, logical indices the identity; a
// position outside [0, L) ([0, H] on a walled z) or a non-finite value sets
// kErrKey.  Store: x[id[j]] = a * stored x[j], likewise v.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_load_f64(Dev d, const double* __restrict__ x,
                                                       const double* __restrict__ v, uint32_t n,
                                                       double a, uint32_t cur) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  BoxRef B = as_const(d.boxes)[0];
  const StatePtrs S = d.S[cur];
  bool ok = true;
  RecF64 r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double xi = x[(uint64_t)k * n + i] / a;
    const double vi = v[(uint64_t)k * n + i] / a;
    const bool in = (B.walls && k == 2) ? (xi >= 0.0 && xi <= B.Ld[k]) : (xi >= 0.0 && xi < B.Ld[k]);
    ok = ok && in && isfinite(vi);
    r.x[k] = in ? xi : 0.0;
    r.v[k] = isfinite(vi) ? vi : 0.0;
  }
  ((RecF64*)S.rec)[i] = r;
  S.id[i] = i;
  if (!ok) atomicOr(&d.ctrl->err, kErrKey);
}

__global__ __launch_bounds__(kThreads) void k_store_f64(Dev d, double* __restrict__ x,
                                                        double* __restrict__ v, uint32_t n,
                                                        double a, uint32_t cur) {
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  const StatePtrs S = d.S[cur];
  const uint32_t l = S.id[j];
  if (l >= n) return;
  const RecF64 r = ((const RecF64*)S.rec)[j];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    x[(uint64_t)k * n + l] = r.x[k] * a;
    v[(uint64_t)k * n + l] = r.v[k] * a;
  }
}

// ---------------------------------------------------------------------------
// Device init: positions uniform, velocities normal (INIT streams keyed by
// the init seed; counter {draw, particle, box, tag}).
// ---------------------------------------------------------------------------
template <int F>
__global__ __launch_bounds__(kThreads) void k_init_state(Dev d, uint32_t k0, uint32_t k1) {
  const PBlock pb = load_pblock(d.pblocks, blockIdx.x);
  BoxRef B = as_const(d.boxes)[pb.box];
  const StatePtrs S = d.S[d.ctrl->cur];
  const uint32_t pend = B.pbase + B.np;
  for (int s = 0; s < kPartBlock / kThreads; ++s) {
    const uint32_t i = pb.p0 + s * kThreads + threadIdx.x;
    if (i >= pend) continue;
    const uint32_t li = i - B.pbase;
    const Words4 a = philox10(0, li, pb.box, kTagInitPos, k0, k1);
    const Words4 b = philox10(1, li, pb.box, kTagInitPos, k0, k1);
    double x[3] = {u53_of(a.w[0], a.w[1]) * B.Ld[0], u53_of(a.w[2], a.w[3]) * B.Ld[1],
                   u53_of(b.w[0], b.w[1]) * B.Ld[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (x[k] >= B.Ld[k]) x[k] = nextafter(B.Ld[k], 0.0);
    const Words4 c = philox10(0, li, pb.box, kTagInitVel, k0, k1);
    const double r0 = sqrt(-2.0 * log(u32_open_of(c.w[0])));
    const double r1 = sqrt(-2.0 * log(u32_open_of(c.w[2])));
    const double t0 = kTwoPi * ((double)c.w[1] * 0x1p-32);
    const double t1 = kTwoPi * ((double)c.w[3] * 0x1p-32);
    const double v[3] = {B.sd * r0 * cos(t0), B.sd * r0 * sin(t0), B.sd * r1 * cos(t1)};
    if constexpr (F == kFormF64) {
      RecF64 r;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        r.x[k] = x[k];
        r.v[k] = v[k];
      }
      ((RecF64*)S.rec)[i] = r;
      S.id[i] = i;
    } else if constexpr (F == kFormF32) {
      RecF32 r;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float xf = (float)x[k];
        if (xf >= B.Lf[k]) xf = nextafterf(B.Lf[k], 0.0f);
        r.x[k] = xf;
        r.v[k] = (float)v[k];
      }
      ((RecF32*)S.rec)[i] = r;
      S.id[i] = i;
    } else {
      RecSplit r;
      int c3[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float o;
        split_from_double(x[k], c3[k], o);
        if (c3[k] >= B.L[k]) {
          c3[k] = B.L[k] - 1;
          o = nextafterf(1.0f, 0.0f);
        }
        r.o[k] = o;
        r.v[k] = (float)v[k];
      }
      r.cell = split_encode(c3);
      r.id = i;
      ((RecSplit*)S.rec)[i] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Observables: per-block partial sums (FP64), reduced on the host side of the
// call in block order.  pass 1: P (3), E; pass 2: sum m |v - vmean|^2.
// ---------------------------------------------------------------------------
template <int F>
__device__ __forceinline__ void load_vel_d(const StatePtrs& S, uint32_t i, double (&v)[3]) {
  if constexpr (F == kFormF64) {
    const RecF64& r = ((const RecF64*)S.rec)[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = r.v[k];
  } else if constexpr (F == kFormF32) {
    const RecF32& r = ((const RecF32*)S.rec)[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = (double)r.v[k];
  } else {
    const RecSplit& r = ((const RecSplit*)S.rec)[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = (double)r.v[k];
  }
}

__device__ __forceinline__ double block_sum_d(double x, double* s_red) {
  // deterministic tree sum over the block (fixed order)
  s_red[threadIdx.x] = x;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_red[threadIdx.x] = s_red[threadIdx.x] + s_red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = s_red[0];
  __syncthreads();
  return r;
}

template <int F>
__global__ __launch_bounds__(kThreads) void k_obs_pass1(Dev d) {
  __shared__ double s_red[kThreads];
  const PBlock pb = load_pblock(d.pblocks, blockIdx.x);
  BoxRef B = as_const(d.boxes)[pb.box];
  const StatePtrs S = d.S[d.ctrl->cur];
  const uint32_t pend = B.pbase + B.np;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < kPartBlock / kThreads; ++s) {
    const uint32_t i = pb.p0 + s * kThreads + threadIdx.x;
    if (i >= pend) continue;
    double v[3];
    load_vel_d<F>(S, i, v);
    acc[0] += B.mass * v[0];
    acc[1] += B.mass * v[1];
    acc[2] += B.mass * v[2];
    acc[3] += 0.5 * B.mass * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  }
  for (int k = 0; k < 4; ++k) {
    const double r = block_sum_d(acc[k], s_red);
    if (threadIdx.x == 0) d.partials[(uint64_t)blockIdx.x * 4 + k] = r;
  }
}

template <int F>
__global__ __launch_bounds__(kThreads) void k_obs_pass2(Dev d, const double* vmean) {
  __shared__ double s_red[kThreads];
  const PBlock pb = load_pblock(d.pblocks, blockIdx.x);
  BoxRef B = as_const(d.boxes)[pb.box];
  const StatePtrs S = d.S[d.ctrl->cur];
  const uint32_t pend = B.pbase + B.np;
  const double V[3] = {vmean[3 * pb.box], vmean[3 * pb.box + 1], vmean[3 * pb.box + 2]};
  double acc = 0.0;
  for (int s = 0; s < kPartBlock / kThreads; ++s) {
    const uint32_t i = pb.p0 + s * kThreads + threadIdx.x;
    if (i >= pend) continue;
    double v[3];
    load_vel_d<F>(S, i, v);
    const double dx = v[0] - V[0], dy = v[1] - V[1], dz = v[2] - V[2];
    acc += B.mass * (dx * dx + dy * dy + dz * dz);
  }
  const double r = block_sum_d(acc, s_red);
  if (threadIdx.x == 0) d.partials[(uint64_t)blockIdx.x * 4] = r;
}

template <int F>
__global__ __launch_bounds__(kThreads) void k_remove_mean(Dev d, const double* vmean) {
  const PBlock pb = load_pblock(d.pblocks, blockIdx.x);
  BoxRef B = as_const(d.boxes)[pb.box];
  const StatePtrs S = d.S[d.ctrl->cur];
  const uint32_t pend = B.pbase + B.np;
  const double V[3] = {vmean[3 * pb.box], vmean[3 * pb.box + 1], vmean[3 * pb.box + 2]};
  for (int s = 0; s < kPartBlock / kThreads; ++s) {
    const uint32_t i = pb.p0 + s * kThreads + threadIdx.x;
    if (i >= pend) continue;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if constexpr (F == kFormF64) {
        double* p = ((RecF64*)S.rec)[i].v;
        p[k] = p[k] - V[k];
      } else if constexpr (F == kFormF32) {
        float* p = ((RecF32*)S.rec)[i].v;
        p[k] = (float)((double)p[k] - V[k]);
      } else {
        float* p = ((RecSplit*)S.rec)[i].v;
        p[k] = (float)((double)p[k] - V[k]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define MPC_FORM_DISPATCH(form, KERNEL, ...)                                  \
  do {                                                                       \
    switch (form) {                                                          \
      case kFormF64: hipLaunchKernelGGL(KERNEL<kFormF64>, __VA_ARGS__); break; \
      case kFormF32: hipLaunchKernelGGL(KERNEL<kFormF32>, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<kFormSplit>, __VA_ARGS__); break;     \
    }                                                                        \
  } while (0)

hipError_t launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s) {
  uint64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_zero_u32, dim3((uint32_t)blocks), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_set_ctrl(const Dev& d, const Launch& l, uint64_t step, uint32_t cur,
                           int32_t reorder, int clear_err) {
  hipLaunchKernelGGL(k_set_ctrl, dim3(1), dim3(1), 0, l.stream, d.ctrl, step, cur, reorder,
                     clear_err);
  return hipGetLastError();
}

hipError_t launch_advance(const Dev& d, const Launch& l) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, l.stream, d.ctrl);
  return hipGetLastError();
}

hipError_t launch_key_hist(const Dev& d, const Launch& l) {
  if (l.npblocks == 0) return hipSuccess;
  const dim3 g(l.npblocks), b(kThreads);
  switch (l.form * 2 + (l.walls ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_key_hist<kFormF64, false>), g, b, 0, l.stream, d); break;
    case 1: hipLaunchKernelGGL((k_key_hist<kFormF64, true>), g, b, 0, l.stream, d); break;
    case 2: hipLaunchKernelGGL((k_key_hist<kFormF32, false>), g, b, 0, l.stream, d); break;
    case 3: hipLaunchKernelGGL((k_key_hist<kFormF32, true>), g, b, 0, l.stream, d); break;
    case 4: hipLaunchKernelGGL((k_key_hist<kFormSplit, false>), g, b, 0, l.stream, d); break;
    default: hipLaunchKernelGGL((k_key_hist<kFormSplit, true>), g, b, 0, l.stream, d); break;
  }
  return hipGetLastError();
}

hipError_t launch_scan(const Dev& d, const Launch& l) {
  hipLaunchKernelGGL(k_scan_reduce, dim3(l.nscan), dim3(kThreads), 0, l.stream, d.hist,
                     d.scan_blk);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, l.stream, d.scan_blk, l.nscan);
  const dim3 g(l.nscan), b(kThreads);
  const uint32_t nb = l.nscan, nx = l.nbox, ct = (uint32_t)l.ctot;
  switch ((l.walls ? 2 : 0) + (l.mbs ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_scan_down<false, false>), g, b, 0, l.stream, d, nb, nx, ct); break;
    case 1: hipLaunchKernelGGL((k_scan_down<false, true>), g, b, 0, l.stream, d, nb, nx, ct); break;
    case 2: hipLaunchKernelGGL((k_scan_down<true, false>), g, b, 0, l.stream, d, nb, nx, ct); break;
    default: hipLaunchKernelGGL((k_scan_down<true, true>), g, b, 0, l.stream, d, nb, nx, ct); break;
  }
  return hipGetLastError();
}

hipError_t launch_phantoms(const Dev& d, const Launch& l) {
  if (!l.walls || l.wcells == 0) return hipSuccess;
  hipLaunchKernelGGL(k_phantom_sums, dim3((l.wcells + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     l.stream, d, l.nbox, l.wcells, l.round_phantoms);
  return hipGetLastError();
}

hipError_t launch_scatter(const Dev& d, const Launch& l) {
  if (l.ntot == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)((l.ntot + kThreads * 4 - 1) / (kThreads * 4));
  hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(kThreads), 0, l.stream, d.key, d.rank,
                     d.offset, d.perm, (uint32_t)l.ntot, (uint32_t)l.ctot, d.ctrl);
  return hipGetLastError();
}

hipError_t launch_collide(const Dev& d, const Launch& l) {
  if (l.ntiles == 0) return hipSuccess;
  return collide_dispatch<CollideLaunchOp>(d, l, nullptr);
}

hipError_t launch_canon_perm(const Dev& d, const Launch& l, const StatePtrs& ids) {
  const uint64_t blocks = (l.ctot + kThreads - 1) / kThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_canon_perm, dim3((uint32_t)blocks), dim3(kThreads), 0, l.stream, d.perm,
                     d.offset, l.ctot, (uint32_t)l.ntot, (const uint32_t*)ids.id, ids.id_stride);
  return hipGetLastError();
}

hipError_t launch_gather_particles(const Dev& d, const Launch& l, const StatePtrs& S,
                                  uint32_t* inv, uint32_t pbase, uint32_t np,
                                  const uint32_t* lidx, uint32_t m, double* out) {
  if (m == 0 || np == 0) return hipSuccess;
  (void)d;
  if (inv) {
    uint64_t blocks = ((uint64_t)np + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_invert_ids, dim3((uint32_t)blocks), dim3(kThreads), 0, l.stream,
                       (const uint32_t*)S.id, S.id_stride, pbase, np, inv);
  }
  MPC_FORM_DISPATCH(l.form, k_gather_particles, dim3((m + kThreads - 1) / kThreads),
                    dim3(kThreads), 0, l.stream, S, inv, pbase, np, lidx, m, out);
  return hipGetLastError();
}

hipError_t launch_load_f64(const Dev& d, const Launch& l, const double* x, const double* v,
                           uint32_t n, double a, uint32_t cur) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_f64, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, l.stream,
                     d, x, v, n, a, cur);
  return hipGetLastError();
}

hipError_t launch_store_f64(const Dev& d, const Launch& l, double* x, double* v, uint32_t n,
                            double a, uint32_t cur) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_store_f64, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     l.stream, d, x, v, n, a, cur);
  return hipGetLastError();
}

hipError_t launch_init_state(const Dev& d, const Launch& l, uint64_t seed) {
  if (l.npblocks == 0) return hipSuccess;
  MPC_FORM_DISPATCH(l.form, k_init_state, dim3(l.npblocks), dim3(kThreads), 0, l.stream, d,
                    (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_obs_pass1(const Dev& d, const Launch& l) {
  if (l.npblocks == 0) return hipSuccess;
  MPC_FORM_DISPATCH(l.form, k_obs_pass1, dim3(l.npblocks), dim3(kThreads), 0, l.stream, d);
  return hipGetLastError();
}

hipError_t launch_obs_pass2(const Dev& d, const Launch& l, const double* vmean) {
  if (l.npblocks == 0) return hipSuccess;
  MPC_FORM_DISPATCH(l.form, k_obs_pass2, dim3(l.npblocks), dim3(kThreads), 0, l.stream, d,
                    vmean);
  return hipGetLastError();
}

hipError_t launch_remove_mean(const Dev& d, const Launch& l, const double* vmean) {
  if (l.npblocks == 0) return hipSuccess;
  MPC_FORM_DISPATCH(l.form, k_remove_mean, dim3(l.npblocks), dim3(kThreads), 0, l.stream, d,
                    vmean);
  return hipGetLastError();
}

}  // namespace mpc
