// Declarations of the mixed-precision (16-bit MFMA + FP32) kernels.
#pragma once
#include <vector>

#include "dp_internal.h"

namespace dpk {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// hi/lo FP16 halves of eight FP32 values x[0..3], y[0..3]: hi = rn16(x),
// lo = rn16(x - hi).  The remainder is rounded in one v_fma_mix{lo,hi}_f16
// per value (FP32 x, FP16 hi operand), two values per register; s_nop 1
// keeps the two wait states a matrix-core read of a VALU-written register
// needs.
__device__ inline unsigned f16_lo_pair(float x, float y, unsigned hi) {
  unsigned lo;
  asm("v_fma_mixlo_f16 %0, %1, 1.0, -%3 op_sel_hi:[0,0,1]\n\t"
      "v_fma_mixhi_f16 %0, %2, 1.0, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
      "s_nop 1"
      : "=&v"(lo)
      : "v"(x), "v"(y), "v"(hi));
  return lo;
}

__device__ inline void split8_f16(const float (&x)[4], const float (&y)[4], f16x8 &hi, f16x8 &lo) {
  typedef _Float16 h2v __attribute__((ext_vector_type(2)));
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const float z[8] = {x[0], x[1], x[2], x[3], y[0], y[1], y[2], y[3]};
  unsigned H[4], L[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const h2v p = {(_Float16)z[2 * k], (_Float16)z[2 * k + 1]};
    H[k] = __builtin_bit_cast(unsigned, p);
    L[k] = f16_lo_pair(z[2 * k], z[2 * k + 1], H[k]);
  }
  const u4v hv = {H[0], H[1], H[2], H[3]}, lv = {L[0], L[1], L[2], L[3]};
  hi = __builtin_bit_cast(f16x8, hv);
  lo = __builtin_bit_cast(f16x8, lv);
}

// tanh(x) = 1 - 2 / (exp(2x) + 1) with the hardware exp2 and reciprocal;
// absolute error about 2e-7, well below the 16-bit storage of the layers.
__device__ inline float tanh_f(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}
// FP64 force of one pair from dE/dR (gr) and the neighbour's displacement
// D4 = (dx, dy, dz, r^2) (neighbours lie within the cut-off, r > 0):
// g = dE/dr_ij (F_i += g, F_j -= g), accumulated into fi and the virial.
// With R = (s, s d / r), s = sw(r) / r and t = s / r = sw / r^2:
//   ds/dr = dsw / r - t,  dt/dr = (dsw / r - 2 t) / r,
//   g = (g0 ds/dr + (g1:3 . d) dt/dr) d / r + t g1:3.
// The switch takes the polynomial at x clamped to [0, 1], which gives
// sw = 1, dsw = 0 inside rcs and sw = 0, dsw = 0 at and beyond rc.
__device__ inline void pair_force(const double4 &D4, float4 gr, double rc, double rcs, double inv_w, double &gx,
                                  double &gy, double &gz, double &fi0, double &fi1, double &fi2, double (&vir)[9]) {
  const double g0 = gr.x, g1 = gr.y, g2 = gr.z, g3 = gr.w;
  const double dx = D4.x, dy = D4.y, dz = D4.z;
  const double ir = rsqrt64(D4.w), r = D4.w * ir;
  const double x = fmin(fmax((r - rcs) * inv_w, 0.0), 1.0);
  const double sw = x * x * x * (-6.0 * x * x + 15.0 * x - 10.0) + 1.0;
  const double dsw = x * x * (-30.0 * x * x + 60.0 * x - 30.0) * inv_w;
  const double ir2 = ir * ir;
  const double tt = sw * ir2;
  const double A = dsw * ir;
  const double ds = A - tt;
  const double dtt = (A - 2.0 * tt) * ir;
  const double gd = g1 * dx + g2 * dy + g3 * dz;
  const double cc = (g0 * ds + dtt * gd) * ir;
  gx = cc * dx + tt * g1;
  gy = cc * dy + tt * g2;
  gz = cc * dz + tt * g3;
  fi0 += gx;
  fi1 += gy;
  fi2 += gz;
  vir[0] -= gx * dx; vir[1] -= gx * dy; vir[2] -= gx * dz;
  vir[3] -= gy * dx; vir[4] -= gy * dy; vir[5] -= gy * dz;
  vir[6] -= gz * dx; vir[7] -= gz * dy; vir[8] -= gz * dz;
}

struct MixArgs {
  Dims d;
  int shape;                  // index into the supported embedding shapes
  int prec;                   // 0 = FP16, 1 = BF16
  const unsigned char *nets;  // packed per-net LDS images, net (t,u) at (t*ntypes+u)*net_bytes
  int64_t rows;
  const int32_t *atom_of_pos;
  const double4 *xw;
  const int32_t *nlist, *nreal;
  const float4 *rt;           // environment matrix rows, FP32
  double L[3];                // box lengths (the force pass recomputes displacements)
  float *T32;                 // [natoms][M1][4], T / Nc (pass 1 writes, pass 2 reads nothing of it)
  const float *dT32;          // [natoms][M1][4], dE/dT of the unscaled sum (pass 2)
  double *force;              // [natoms][3]
  double *vir_part;           // [grid][9]
  double *net_deriv;          // optional [natoms][nnei][4]
  // tabulated second layer of a student net (NULL: evaluate the layers):
  // per net [TAB_K + 1][TAB_STRIDE] floats, row k = s_k = k ds, features f
  // at (2f, 2f+1) = (h2(s_k), ds dh2/ds(s_k)); s above tab_shi takes the
  // layers themselves
  const float *tab;
  float tab_inv_ds, tab_shi;
  // with tab: the backward's projected-table operands (launch_student_pimg),
  // and the nets it leaves to the layers (a neighbour beyond the table's
  // range): entries i * ntypes + u, their count zeroed before the backward
  const unsigned char *pimg;
  int32_t *defer;
  uint32_t *defer_count;
};

constexpr int TAB_K = 80;                         // intervals of the student table
constexpr int TAB_STRIDE = 68;                    // floats per row: 32 features x 2 + 4 (LDS bank spread)
constexpr int TAB_BYTES = (TAB_K + 1) * TAB_STRIDE * 4;
// second layer of each student net tabulated (cubic Hermite data) over [0, shi]
void launch_student_table(hipStream_t s, const Dims &d, const EmbOffsets &eo, const double *ew, int prec, double shi,
                          float *tab);
// The student backward contracts the table with M = W3 dT per (atom, net):
// rows (y_k, y_{k+1} - y_k, m_k) of the TAB_K + 1 nodes, PT_TILES MFMA tiles
// of 16 rows; per net an image of PT_TILES x (hi, lo) 1 KB operand blocks,
// per wave PT_BYTES of LDS for the projected rows (float4 each)
constexpr int PT_TILES = 16;
constexpr int PIMG_BYTES = PT_TILES * 2 * 1024;
constexpr int PT_BYTES = PT_TILES * 16 * 16;
static_assert(3 * (TAB_K + 1) <= 16 * PT_TILES, "projected rows must fit the tiles");
void launch_student_pimg(hipStream_t s, int nets, const float *tab, int prec, unsigned char *img);
// largest s of the frame (nearest neighbour of every atom and type) into *smax (bits of a float)
void launch_smax(hipStream_t s, int64_t n, const Dims &d, const int32_t *nreal, const float4 *rt, uint32_t *smax);

int mix_shape_id(const Dims &d);
size_t mix_net_bytes(int shape);
bool mix_tab_fits(int shape, int ntypes);  // affine-net kernels fit the LDS with the student table
size_t mix_lds_bytes(int shape, int ntypes, int pass);
void mix_pack_net(int shape, const double *const *W, const double *const *b, int prec, unsigned char *out);
int mix_grid(int64_t rows);
void launch_embed_mix(hipStream_t s, const MixArgs &a, int pass, int grid);
// the deferred nets of a table backward, by the layers (grid DEFER_GRID;
// virial partials in a.vir_part[0 .. DEFER_GRID))
constexpr int DEFER_GRID = 64;
void launch_embed_defer(hipStream_t s, const MixArgs &a);

// fused fitting net: byte offsets of the per-type operand images
struct FitMixOffsets {
  int64_t a0f[MAXT];            // layer 0 forward A operands (W0^T, D-slot order)
  int64_t a0b[MAXT];            // layer 0 backward A operands (W0, chained order)
  int64_t ahf[MAXT][MAXF];      // hidden layer l >= 1 forward (W^T)
  int64_t ahf_lo[MAXT][MAXF];   // rounding remainders of ahf (layers >= nsplit)
  int64_t ahb[MAXT][MAXF];      // hidden layer l >= 1 backward (W)
  int64_t ahb_lo[MAXT][MAXF];
  int64_t bias[MAXT][MAXF];     // f32 [256] per hidden layer
  int64_t wout[MAXT];           // f32 [256] output weights, [256] = output bias
};

struct FitMixArgs {
  Dims d;
  FitMixOffsets fo;
  const unsigned char *w;
  int prec;                   // 0 = FP16, 1 = BF16
  int nsplit;                 // hidden layers >= nsplit carry hi + lo weights
  const int32_t *type_start;
  const int32_t *atom_of_pos;
  int64_t rows;
  const float *T32;           // [natoms][M1][4] (T / Nc)
  float *tbuf;                // tanh outputs per 16-row tile
  float *dT32;                // [natoms][M1][4] output of pass 2
  double *eatom;              // [natoms] output of pass 1
  float inv_nc;
};

// cell-ordered backward of the affine-last-layer nets (k_embed_bwd_cells)
constexpr int CELL_WAVES = 16;   // waves per workgroup at most
// with the table at most 12 (three per SIMD, up to 168 registers each): the
// projection images take the LDS a fourth wave per SIMD would need
__host__ __device__ constexpr int cell_waves(bool proj) { return proj ? 12 : CELL_WAVES; }
constexpr int CELL_CAP = 128;    // atoms per cell kept in LDS; the rest use global atomics
struct CellArgs {
  const int32_t *cell_start;     // [ncell + 1]
  const int32_t *cell_atoms;     // [n] atoms in cell order
  const int32_t *cell_of;        // [n]
  const uint32_t *code;          // [n] cx << 24 | cy << 16 | cz << 8 | min(index in cell, 255)
  int nc[3];
  int cap;
  int64_t ncell, n;
  double *part;                  // [27][n][3] per-cell parts of the forces, cell order
};
// accumulator capacity (atoms per cell, need <= cap <= want), workgroup size
// and LDS bytes of the cell kernel: the most waves that leave room for at
// least `need` atoms per cell; false when the net shape or the LDS budget
// does not allow it
bool embed_cells_config(const MixArgs &a, int want, int need, int *cap, int *threads, size_t *lds);
int cells_grid(int64_t ncell);
void launch_embed_cells(hipStream_t s, const MixArgs &a, const CellArgs &ca, int grid, int threads, size_t lds);
void launch_cell_gather(hipStream_t s, const CellArgs &ca, double *F);

bool fit_mix_supported(const Dims &d, const char **why);
void fit_mix_pack(const Dims &d, int prec, int nsplit, const double *const *W, const double *const *b,
                  std::vector<unsigned char> &buf, FitMixOffsets &fo);
size_t fit_mix_tbuf_floats(const Dims &d, int64_t rows);
// pass 1: forward layers and E_i; pass 2: backward to dE/dT
void launch_fit_mix(hipStream_t s, const FitMixArgs &a, int pass);

}  // namespace dpk
