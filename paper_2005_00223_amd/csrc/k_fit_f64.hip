// Double-precision fitting net, forward and backward, per centre type
// (Fig. 1(d,g)).  Rows are atoms in the type-padded row order (each type's
// rows padded to ROW_TILE, so a 64-row tile never mixes types).
//
// Forward hidden layer l (in -> out):  t = tanh(Y_l W + b),
//   Y_{l+1} = t (+ Y_l if out == in, + (Y_l, Y_l) if out == 2 in).
// The bias add, tanh, skip add and the store of t (kept for the backward,
// the paper's fused TANH/TANHGrad idea) all sit in the GEMM epilogue
// (Section V-C, "Replace MATMUL and SUM" and "Replace CONCAT and SUM").
// Output layer: E_i = Y_L . w + b (one wave per row).
// Backward layer l: gZ = gY_{l+1} (1 - t^2) is formed while the A tile is
// loaded, gY_l = gZ W^T (+ the skip's pass-through), gY_0 = dE/dD.
//
// MFMA v_mfma_f64_16x16x4 (D register r of lane l is row 4r + l/16,
// column l%16), or v_mfma_f32_16x16x4_f32 for DP_MIX_FP32 (row 4(l/16) + r);
// block tile 64 x 64, four waves of 32 x 32, K staged through LDS in steps
// of 16.  The per-atom energies are written in double either way.
//
// Block order: the column blocks of one 64-row block run back to back on
// one XCD (workgroups are dealt to the eight XCDs round-robin by linear id),
// so the row block's A tiles -- D in the forward's first layer (1600
// columns), the tanh outputs and incoming gradient in the backward's
// (25 column blocks of the 1600 outputs) -- come from HBM once and from
// that XCD's L2 for the other column blocks.
#include "dp_f64.h"

namespace dpk {

constexpr int BM = 64, BN = 64, BK = 16, APAD = BK + 1;

enum { FIT_FWD = 0, FIT_BWD = 1 };

template <typename Real>
struct GemmArgs {
  int mode, layer, K, N, in, out;  // in/out of the layer (fwd: K=in, N=out; bwd: K=out, N=in)
  int ntypes;
  int64_t nrb;                      // 64-row blocks
  const int32_t *type_start;
  const Real *fwt;
  FitOffsets fo;
  const Real *X;    // fwd: layer input [rows][in]
  Real *Tt;         // fwd: tanh output [rows][out] (written); bwd: read
  Real *Y;          // fwd: layer output [rows][out]
  const Real *gY;   // bwd: gradient wrt the layer output [rows][out] (NULL = output weights)
  const Real *wout; // bwd: output-layer weights of each type when gY == NULL (offset by type)
  Real *gX;         // bwd: gradient wrt the layer input [rows][in]
};

__device__ inline int row_type(const int32_t *ts, int ntypes, int64_t r0) {
  int t = 0;
  for (int u = 1; u < ntypes; ++u)
    if (r0 >= ts[u]) t = u;
  return t;
}

template <int MODE, typename Real>
__global__ void __launch_bounds__(256) k_fit_gemm(GemmArgs<Real> g) {
  __shared__ Real As[BM][APAD];
  __shared__ Real Bs[BK][BN];
  const int gn = (g.N + BN - 1) / BN;
  const unsigned q = blockIdx.x >> 3;
  const int64_t rb = (int64_t)(q / gn) * 8 + (blockIdx.x & 7);
  const int64_t r0 = rb * BM;
  const int c0 = (int)(q % gn) * BN;
  if (rb >= g.nrb || r0 >= g.type_start[g.ntypes]) return;
  const int t = row_type(g.type_start, g.ntypes, r0);
  const Real *W = g.fwt + g.fo.w[t][g.layer];
  const Real *bias = g.fwt + g.fo.b[t][g.layer];
  const Real *wo = (MODE == FIT_BWD && g.gY == nullptr) ? g.fwt + g.fo.w[t][g.layer + 1] : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  typename MF<Real>::acc acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = typename MF<Real>::acc{0, 0, 0, 0};

  // the next K-tile's global loads are issued before the current tile's
  // products and stored to LDS after them (raw values: the backward forms
  // gy (1 - t^2) at the store)
  Real xa[4], xb[4], xw[4];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int rr = e >> 4, k = k0 + (e & 15);
      const int64_t row = r0 + rr;
      xa[q] = 0;
      xb[q] = 0;
      if (k < g.K) {
        if (MODE == FIT_FWD) {
          xa[q] = g.X[row * g.K + k];
        } else {
          xa[q] = g.Tt[row * g.K + k];
          xb[q] = wo ? wo[k] : g.gY[row * g.K + k];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int k = k0 + (e >> 6), c = c0 + (e & 63);
      xw[q] = 0;
      if (k < g.K && c < g.N) xw[q] = (MODE == FIT_FWD) ? W[(int64_t)k * g.N + c] : W[(int64_t)c * g.K + k];
    }
  };
  load_tile(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // A tile [64 x 16], B tile [16 x 64]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      As[e >> 4][e & 15] = MODE == FIT_FWD ? xa[q] : xb[q] * (Real(1) - xa[q] * xa[q]);
      Bs[e >> 6][e & 63] = xw[q];
    }
    __syncthreads();
    if (k0 + BK < g.K) load_tile(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      Real af[2], bf[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) af[mi] = As[wm * 32 + mi * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) bf[ni] = Bs[ks + (lane >> 4)][wn * 32 + ni * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = MF<Real>::mma(af[mi], bf[ni], acc[mi][ni]);
    }
    __syncthreads();
  }
  // epilogue
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + mi * 16 + MF<Real>::row(r, lane >> 4);
        const int col = c0 + wn * 32 + ni * 16 + (lane & 15);
        if (col >= g.N) continue;
        const Real c = acc[mi][ni][r];
        if (MODE == FIT_FWD) {
          const Real th = MF<Real>::tanh_(c + bias[col]);
          Real y = th;
          if (g.out == g.in) y += g.X[row * g.in + col];
          else if (g.out == 2 * g.in) y += g.X[row * g.in + (col >= g.in ? col - g.in : col)];
          g.Tt[row * g.out + col] = th;
          g.Y[row * g.out + col] = y;
        } else {
          Real v = c;
          if (g.out == g.in || g.out == 2 * g.in) {
            v += wo ? wo[col] : g.gY[row * g.out + col];
            if (g.out == 2 * g.in) v += wo ? wo[col + g.in] : g.gY[row * g.out + col + g.in];
          }
          g.gX[row * g.in + col] = v;
        }
      }
}

// E_i = Y_L . w_out + b_out, one wave per row (in Real, stored as double)
template <typename Real>
__global__ void __launch_bounds__(256) k_fit_out(const int32_t *type_start, int ntypes, const int32_t *atom_of_pos,
                                                 const Real *fwt, FitOffsets fo, int L, int width, const Real *Y,
                                                 int64_t rows_cap, double *eatom) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_cap || row >= type_start[ntypes]) return;
  const int atom = atom_of_pos[row];
  if (atom < 0) return;
  const int t = row_type(type_start, ntypes, row);
  const Real *w = fwt + fo.w[t][L];
  Real s = 0;
  for (int o = lane; o < width; o += 64) s += Y[row * width + o] * w[o];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) eatom[atom] = (double)(s + fwt[fo.b[t][L]]);
}

// blocks of the XCD-grouped order: row blocks rounded up to a multiple of
// eight, times the column blocks
static unsigned fit_blocks(unsigned gm, int n) {
  return ((gm + 7u) / 8u) * 8u * (unsigned)((n + BN - 1) / BN);
}

template <typename Real>
static void launch_fit_t(hipStream_t s, const FitArgsT<Real> &a, int pass) {
  const Dims &d = a.d;
  const int L = d.n_fit;
  const unsigned gm = (unsigned)((a.rows + BM - 1) / BM);
  for (int l = 0; l < L && pass == 1; ++l) {
    GemmArgs<Real> g{};
    g.mode = FIT_FWD;
    g.layer = l;
    g.in = d.fw[l];
    g.out = d.fw[l + 1];
    g.K = g.in;
    g.N = g.out;
    g.ntypes = d.ntypes;
    g.type_start = a.type_start;
    g.fwt = a.fwt;
    g.fo = a.fo;
    g.X = (l == 0) ? a.X0 : a.Y[l];
    g.Tt = a.Tt[l + 1];
    g.Y = a.Y[l + 1];
    g.nrb = gm;
    hipLaunchKernelGGL((k_fit_gemm<FIT_FWD, Real>), dim3(fit_blocks(gm, g.N)), dim3(256), 0, s, g);
  }
  if (pass == 1)
    hipLaunchKernelGGL(k_fit_out<Real>, dim3((unsigned)((a.rows + 3) / 4)), dim3(256), 0, s, a.type_start, d.ntypes,
                       a.atom_of_pos, a.fwt, a.fo, L, d.fw[L], a.Y[L], a.rows, a.eatom);
  for (int l = L - 1; l >= 0 && pass == 2; --l) {
    GemmArgs<Real> g{};
    g.mode = FIT_BWD;
    g.layer = l;
    g.in = d.fw[l];
    g.out = d.fw[l + 1];
    g.K = g.out;
    g.N = g.in;
    g.ntypes = d.ntypes;
    g.type_start = a.type_start;
    g.fwt = a.fwt;
    g.fo = a.fo;
    g.Tt = a.Tt[l + 1];
    g.gY = (l == L - 1) ? nullptr : a.G[l + 1];
    g.gX = a.G[l];
    g.nrb = gm;
    hipLaunchKernelGGL((k_fit_gemm<FIT_BWD, Real>), dim3(fit_blocks(gm, g.N)), dim3(256), 0, s, g);
  }
}

void launch_fit_f64(hipStream_t s, const FitArgs &a, int pass) { launch_fit_t<double>(s, a, pass); }
void launch_fit_f32(hipStream_t s, const FitArgs32 &a, int pass) { launch_fit_t<float>(s, a, pass); }

}  // namespace dpk
