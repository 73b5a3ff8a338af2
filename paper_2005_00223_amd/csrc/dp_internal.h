// Internal declarations shared by the host runtime (api.cpp) and the HIP
// kernels of the Deep Potential evaluator.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dpk {

constexpr int MAXT = 8;        // atom types
constexpr int MAXL = 4;        // embedding layers
constexpr int MAXF = 4;        // hidden fitting layers
constexpr int KEY_CAP = 512;   // neighbours within rc per atom held by the LDS sort
constexpr int ROW_TILE = 128;  // fitting-net row tile; each type's rows are padded to it

// Geometry / model dimensions passed by value to every kernel.
struct Dims {
  int ntypes, n_emb, n_fit, M1, M2, nnei;
  double rcut, rcut_smth, inv_nc;
  int sel[MAXT], off[MAXT + 1];
  int ew[MAXL + 1];    // embedding widths, ew[0] = 1
  int ekp[MAXL + 1];   // width rounded up to 4 (as a K dimension)
  int emp[MAXL + 1];   // width rounded up to 16 (as an M dimension)
  int emb_lin;         // 1: the last embedding layer is affine (no tanh)
  int fw[MAXF + 2];    // fitting widths, fw[0] = M1*M2, fw[n_fit+1] = 1
};

// Offsets (in elements) of the padded embedding weights inside one flat
// array.  Layer 0 (1 -> ew[1]) is stored as W0[ekp[1]], b0[ekp[1]]; layer
// l >= 1 as W[ekp[l]][emp[l+1]] (row = input feature), b[emp[l+1]], zero
// padded.  One net per (centre type t, neighbour type u).
struct EmbOffsets {
  int64_t w[MAXT][MAXT][MAXL];
  int64_t b[MAXT][MAXT][MAXL];
};

// Offsets of the fitting weights: layer l of type t, W[fw[l]][fw[l+1]]
// row-major (input feature = row), b[fw[l+1]].  Output layer is l = n_fit.
struct FitOffsets {
  int64_t w[MAXT][MAXF + 1];
  int64_t b[MAXT][MAXF + 1];
};

// Error flags written by kernels, read back by the host.
enum : uint32_t { FLAG_BAD_TYPE = 1u, FLAG_CAND_CAP = 2u, FLAG_KEY_CAP = 4u, FLAG_NONFINITE = 8u,
                  FLAG_REBUILD = 16u };
// Flags that stop an MD run: once one is set, the integrator kernels leave
// coordinates and velocities as they are until the host reads the flags.
constexpr uint32_t FLAG_HALT = FLAG_BAD_TYPE | FLAG_CAND_CAP | FLAG_KEY_CAP | FLAG_NONFINITE;

struct NlistBufs {
  const double *coords;  // caller coords [n][3]
  const int32_t *types;  // caller types [n]
  double4 *xw;           // wrapped coords, w = type
  int32_t *cell_of;      // [n]
  int32_t *cell_start;   // [ncell + 1]
  int32_t *cell_fill;    // [ncell]
  int32_t *cell_atoms;   // [n]
  int32_t *cand;         // [n][cand_cap]
  int32_t *cand_n;       // [n]
  int32_t *nlist;        // [n][nnei]
  int32_t *nreal;        // [n][ntypes]
  unsigned long long *overflow;  // [1]
  int32_t *max_real;     // [MAXT]
  uint32_t *flags;       // [1]
};

struct CellGrid {
  int nc[3];
  double side[3];
  double L[3];
};

// ---- neighbour list (k_nlist.hip) ----
void launch_wrap(hipStream_t s, int64_t n, const double *coords, const int32_t *types, int ntypes,
                 const double *L, double4 *xw, uint32_t *flags);
// mask (may be NULL): rows only for atoms with mask[i] != 0; pos_of_atom may be NULL
void launch_type_sort(hipStream_t s, int64_t n, const double4 *xw, int ntypes, int32_t *blk_counts,
                      int32_t *type_count, int32_t *type_start, int32_t *pos_of_atom, int32_t *atom_of_pos,
                      int64_t rows_cap, const int32_t *mask = nullptr);
// `cond` (may be NULL): when given, the kernels do nothing unless
// (*cond & FLAG_REBUILD) -- the MD driver decides on the device.
// cell_code (may be NULL): per-atom cell coordinates and index inside the cell
void launch_cells(hipStream_t s, int64_t n, const double4 *xw, const CellGrid &g, int32_t *cell_of,
                  int32_t *cell_start, int32_t *cell_fill, int32_t *cell_atoms, uint32_t *cell_code,
                  int32_t *scan_tmp, const uint32_t *cond);
void launch_candidates(hipStream_t s, int64_t n, const double4 *xw, const CellGrid &g, const int32_t *cell_start,
                       const int32_t *cell_atoms, double rlist, int cand_cap, int32_t *cand, int32_t *cand_n,
                       uint32_t *flags, const uint32_t *cond);
void launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t v);
// rt32 (may be NULL): also write the mixed path's FP32 environment rows of
// the real slots (then the environment kernel is not needed)
void launch_format(hipStream_t s, int64_t n, const double4 *xw, const Dims &d, const double *L, const int32_t *cand,
                   const int32_t *cand_n, int cand_cap, int32_t *nlist, int32_t *nreal,
                   unsigned long long *overflow, int32_t *max_real, uint32_t *flags, float4 *rt32);
// -1 padding of the formatted list past each type's real count (the
// formatting kernel writes the real slots only)
void launch_pad_nlist(hipStream_t s, int64_t n, const Dims &d, const int32_t *nreal, int32_t *nlist);
void launch_max_disp(hipStream_t s, int64_t n, const double4 *xw, const double4 *xref, const double *L,
                     double half_skin, uint32_t *flags);
void launch_copy_ref(hipStream_t s, int64_t n, const double4 *xw, double4 *xref, const uint32_t *cond);
// clears FLAG_REBUILD and counts the rebuild in *nbuild when it was set
void launch_end_rebuild(hipStream_t s, uint32_t *flags, unsigned long long *nbuild);

// ---- environment matrix (k_env.hip) ----
// s(r) = sw(r) / r with the quintic switch, FP64; the one expression both the
// environment kernel and the student sampler evaluate
__device__ inline double env_s(double r, double rcs, double rc, double inv_w) {
  double sw;
  if (r < rcs) {
    sw = 1.0;
  } else if (r < rc) {
    const double x = (r - rcs) * inv_w;
    sw = x * x * x * (-6.0 * x * x + 15.0 * x - 10.0) + 1.0;
  } else {
    sw = 0.0;
  }
  return sw * (1.0 / r);
}
// displacement d = x_j - x_i (one minimum-image correction per axis) and
// r = |d| of a pair from the wrapped positions: (dx, dy, dz, r)
__device__ inline double4 pair_disp(const double4 &pi, const double4 &pj, double L0, double L1, double L2) {
  double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
  if (dx > 0.5 * L0) dx -= L0;
  else if (dx < -0.5 * L0) dx += L0;
  if (dy > 0.5 * L1) dy -= L1;
  else if (dy < -0.5 * L1) dy += L1;
  if (dz > 0.5 * L2) dz -= L2;
  else if (dz < -0.5 * L2) dz += L2;
  return make_double4(dx, dy, dz, sqrt(dx * dx + dy * dy + dz * dz));
}
// nearest image of a coordinate difference d (|d| < 1.5 L) as selects: the
// values of the branch form above, without branches around the pair's work
__device__ inline double min_img_sel(double d, double L) {
  const double h = 0.5 * L, up = d - L, dn = d + L;
  return d > h ? up : (d < -h ? dn : d);
}
// the same displacement with r^2 in place of r: (dx, dy, dz, r^2)
__device__ inline double4 pair_disp_sq(const double4 &pi, const double4 &pj, double L0, double L1, double L2) {
  const double dx = min_img_sel(pj.x - pi.x, L0), dy = min_img_sel(pj.y - pi.y, L1),
               dz = min_img_sel(pj.z - pi.z, L2);
  return make_double4(dx, dy, dz, dx * dx + dy * dy + dz * dz);
}
// tanh in FP64 to a few ulp, about a fifth of the instructions of the
// library routine (which carries double-double intermediates):
//   tanh|x| = -m / (2 + m),  m = expm1(-2|x|) in (-1, 0],
// expm1 by Cody and Waite's argument reduction z = k ln2 + r (|r| <= ln2/2,
// ln2 as a double plus its remainder) and the Taylor series of expm1(r) to
// r^13 (remainder below 2^-56 relative), expm1(z) = 2^k expm1(r) + (2^k - 1);
// the quotient by a Newton-refined hardware reciprocal with one residual
// correction.  |x| is capped at 20, where tanh rounds to 1; NaN stays NaN.
__device__ inline double tanh64(double x) {
  double a = fabs(x);
  a = a > 20.0 ? 20.0 : a;
  const double z = -2.0 * a;
  const double kd = rint(z * 1.4426950408889634);  // z / ln2
  double r = fma(-kd, 0.6931471805599453, z);
  r = fma(-kd, 2.3190468138462996e-17, r);
  double q = 1.0 / 6227020800.0;  // 1/13!
  q = fma(q, r, 1.0 / 479001600.0);
  q = fma(q, r, 1.0 / 39916800.0);
  q = fma(q, r, 1.0 / 3628800.0);
  q = fma(q, r, 1.0 / 362880.0);
  q = fma(q, r, 1.0 / 40320.0);
  q = fma(q, r, 1.0 / 5040.0);
  q = fma(q, r, 1.0 / 720.0);
  q = fma(q, r, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  const double p = q * r;  // expm1(r)
  const double sk = ldexp(1.0, (int)kd);
  const double m = fma(sk, p, sk - 1.0);
  const double den = 2.0 + m, num = -m;
  double y = __builtin_amdgcn_rcp(den);
  double e = fma(-den, y, 1.0);
  y = fma(y, e, y);
  e = fma(-den, y, 1.0);
  y = fma(y, e, y);
  double t = num * y;
  t = fma(fma(-den, t, num), y, t);
  return copysign(t, x);
}
// 1/sqrt(x) for normal x > 0: the hardware estimate (relative error below
// 2^-22) and two Newton steps y += y (1 - x y^2) / 2, each squaring the
// relative error, which leaves a few ulp of FP64
__device__ inline double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
// exactly one of rt (FP64 evaluation) and rt32 (mixed precision, the same
// values rounded to FP32, which is all the mixed kernels read) is non-NULL;
// dr (may be NULL: the mixed kernels recompute it from the positions)
void launch_env(hipStream_t s, int64_t n, const double4 *xw, const Dims &d, const double *L, const int32_t *nlist,
                const int32_t *nreal, double4 *rt, float4 *rt32, double4 *dr);

// ---- FP64 / FP32 embedding + descriptor (k_embed_f64.hip) ----
// Real = double (DP_FP64) or float (DP_MIX_FP32: weights, R, T, D and dE/dD
// in FP32; displacements, the force Jacobian, forces and the virial in FP64)
template <typename Real, typename Real4>
struct EmbedArgsT {
  Dims d;
  EmbOffsets eo;
  const Real *ew;            // padded embedding weights
  const int32_t *atom_of_pos;
  const int32_t *pos_of_atom;
  const int32_t *type_start; // [ntypes+1] padded row starts
  int64_t rows;              // padded rows in use
  int64_t natoms;
  const double4 *xw;
  const int32_t *nlist, *nreal;
  const Real4 *rt;           // environment rows
  const double4 *dr;         // displacements (dx, dy, dz, r)
  Real *T;                   // [natoms][M1][4]
  Real *D;                   // [rows][M1*M2]
  const Real *dD;            // [rows][M1*M2]
  double *force;             // [natoms][3]
  double *vir_part;          // [grid][9]
  double *net_deriv;         // optional [natoms][nnei][4]
};
typedef EmbedArgsT<double, double4> EmbedArgs;
typedef EmbedArgsT<float, float4> EmbedArgs32;
void launch_embed_fwd_f64(hipStream_t s, const EmbedArgs &a);
void launch_embed_bwd_f64(hipStream_t s, const EmbedArgs &a, int grid);
void launch_embed_fwd_f32(hipStream_t s, const EmbedArgs32 &a);
void launch_embed_bwd_f32(hipStream_t s, const EmbedArgs32 &a, int grid);
int embed_bwd_grid(int64_t rows);

// ---- FP64 / FP32 fitting net (k_fit_f64.hip) ----
template <typename Real>
struct FitArgsT {
  Dims d;
  FitOffsets fo;
  const Real *fwt;            // fitting weights
  const int32_t *type_start;  // [ntypes+1] padded row starts (device)
  const int32_t *atom_of_pos; // [rows]
  int64_t rows;
  Real *X0;                   // D [rows][fw0]
  Real *Y[MAXF + 1];          // Y[l] l=1..n_fit [rows][fw[l]]
  Real *Tt[MAXF + 1];         // tanh outputs per layer [rows][fw[l]]
  Real *G[MAXF + 1];          // gradient wrt Y[l] [rows][fw[l]]; G[0] = dD
  double *eatom;              // [natoms] (original order)
};
typedef FitArgsT<double> FitArgs;
typedef FitArgsT<float> FitArgs32;
// pass 1: forward layers and E_i; pass 2: backward to dE/dD
void launch_fit_f64(hipStream_t s, const FitArgs &a, int pass);
void launch_fit_f32(hipStream_t s, const FitArgs32 &a, int pass);

// ---- reductions and MD (k_md.hip) ----
void launch_sum(hipStream_t s, const double *x, int64_t n, double *partial, double *out, double scale);
void launch_sum9(hipStream_t s, const double *part, int nparts, double *out);
void launch_zero(hipStream_t s, double *x, int64_t n);
// Half kick v += half_dt F / m.  Skipped when *flags holds a FLAG_HALT bit;
// the first skipped kick stores `step` in *fault_step (when it is < 0).
void launch_verlet_half(hipStream_t s, int64_t n, double *v, const double *f, const int32_t *types,
                        const double *inv_m_conv, double half_dt, const uint32_t *flags, long long *fault_step,
                        int64_t step);
// Drift x += dt v and wrap; skipped when *flags holds a FLAG_HALT bit.
void launch_verlet_drift(hipStream_t s, int64_t n, double *x, const double *v, double dt, const double *L,
                         const uint32_t *flags);
void launch_kinetic(hipStream_t s, int64_t n, const double *v, const int32_t *types, const double *mass,
                    double *partial, double *out);
void launch_thermo_row(hipStream_t s, double *row, double step, const double *ke, const double *pe,
                       const double *vir, double ndof_kb, double inv3v, uint32_t *flags);

}  // namespace dpk
