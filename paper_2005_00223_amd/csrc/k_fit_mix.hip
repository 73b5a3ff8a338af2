// Mixed-precision fitting net (Fig. 1(d,g); Section V-A "Mixed-precision
// computation"): the first two hidden layers are 16-bit matrix-core GEMMs
// (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulation, 16-bit weights), the
// remaining hidden layers and the output layer run in FP32
// (v_mfma_f32_16x16x4f32), tanh and the skip adds in FP32; E_i is converted
// to FP64 before the reduction.  Backward mirrors it; dE/dD leaves in FP32.
// The activation operand of each 16-bit GEMM is split into hi + lo 16-bit
// parts on its way into LDS and multiplied twice, so only the weights are
// rounded to 16 bits.
//
// Tiles: 64 rows x 64 columns per 256-thread block, four waves of 32 x 32.
// 16-bit: K steps of 32 staged in LDS as [row][k] (A hi and lo) and [col][k]
// (B, from a W^T copy in the forward and from W itself in the backward) with
// a padded row stride of 40 elements, so each lane's eight K values are one
// conflict-free 16-byte LDS read.
#include <cstring>

#include "dp_mix.h"

namespace dpk {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int P> struct FT;
template <> struct FT<0> {
  typedef _Float16 e;
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  __device__ static v4f mma(v8 a, v8 b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <> struct FT<1> {
  typedef __bf16 e;
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  __device__ static v4f mma(v8 a, v8 b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

__device__ inline float ftanh(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ inline int rtype(const int32_t *ts, int ntypes, int64_t r0) {
  int t = 0;
  for (int u = 1; u < ntypes; ++u)
    if (r0 >= ts[u]) t = u;
  return t;
}

enum { MF_FWD = 0, MF_BWD = 1 };

struct MG {
  int layer, K, N, in, out, ntypes, last_hidden;
  const int32_t *type_start;
  const unsigned char *w;
  FitMixOffsets fo;
  const float *Xf;     // fwd: f32 input [rows][K] (also the skip source)
  float *Tt;           // tanh out [rows][out]
  float *Y;            // f32 out [rows][out]
  const float *gY;     // bwd: dE/dY_out [rows][out]; NULL -> output weights
  float *gX;           // bwd: dE/dY_in [rows][in]
};

constexpr int TS = 40;  // padded LDS row stride (elements) for 16-bit tiles

template <int P, int MODE>
__global__ void __launch_bounds__(256) k_fitmix16(MG g) {
  typedef typename FT<P>::e E;
  typedef typename FT<P>::v8 V;
  __shared__ __align__(16) E Ah[64 * TS];
  __shared__ __align__(16) E Al[64 * TS];
  __shared__ __align__(16) E Bs[64 * TS];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  if (r0 >= g.type_start[g.ntypes]) return;
  const int t = rtype(g.type_start, g.ntypes, r0);
  const E *Bt = (const E *)(g.w + (MODE == MF_FWD ? g.fo.wt16[t][g.layer] : g.fo.w16[t][g.layer]));
  const float *bias = (const float *)(g.w + g.fo.b32[t][g.layer]);
  const float *wo = (MODE == MF_BWD && g.gY == nullptr) ? (const float *)(g.w + g.fo.w32[t][g.layer + 1]) : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  v4f acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = v4f{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 2, lk = (tid & 3) * 8;  // tile loader: row (or col) and 8-wide k chunk
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    const int k = k0 + lk;
    // A tile [64 rows][32 k], split into hi + lo
    {
      float x[8];
      const int64_t row = r0 + lr;
      if (k < g.K) {
        if (MODE == MF_FWD) {
          const float4 *xp = (const float4 *)(g.Xf + row * g.K + k);
          const float4 a0 = xp[0], a1 = xp[1];
          x[0] = a0.x; x[1] = a0.y; x[2] = a0.z; x[3] = a0.w;
          x[4] = a1.x; x[5] = a1.y; x[6] = a1.z; x[7] = a1.w;
        } else {
          const float4 *tp = (const float4 *)(g.Tt + row * g.K + k);
          const float4 t0 = tp[0], t1 = tp[1];
          const float4 *gp = (const float4 *)(wo ? wo + k : g.gY + row * g.K + k);
          const float4 a0 = gp[0], a1 = gp[1];
          const float gy[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
          const float th[8] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) x[q] = gy[q] * (1.f - th[q] * th[q]);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = 0.f;
      }
      V hi, lo;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const E h = (E)x[q];
        hi[q] = h;
        lo[q] = (E)(x[q] - (float)h);
      }
      *(V *)(Ah + lr * TS + lk) = hi;
      *(V *)(Al + lr * TS + lk) = lo;
    }
    // B tile as [64 cols][32 k] from Bt [N][K]
    {
      V v;
      const int col = c0 + lr;
      if (k < g.K && col < g.N) {
        v = *(const V *)(Bt + (int64_t)col * g.K + k);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (E)0.f;
      }
      *(V *)(Bs + lr * TS + lk) = v;
    }
    __syncthreads();
    V ah[2], al[2], bf[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int o = (wm * 32 + mi * 16 + (lane & 15)) * TS + 8 * (lane >> 4);
      ah[mi] = *(const V *)(Ah + o);
      al[mi] = *(const V *)(Al + o);
    }
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) bf[ni] = *(const V *)(Bs + (wn * 32 + ni * 16 + (lane & 15)) * TS + 8 * (lane >> 4));
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        acc[mi][ni] = FT<P>::mma(ah[mi], bf[ni], acc[mi][ni]);
        acc[mi][ni] = FT<P>::mma(al[mi], bf[ni], acc[mi][ni]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + r;
        const int col = c0 + wn * 32 + ni * 16 + (lane & 15);
        if (col >= g.N) continue;
        const float c = acc[mi][ni][r];
        if (MODE == MF_FWD) {
          const float th = ftanh(c + bias[col]);
          float y = th;
          if (g.out == g.in) y += g.Xf[row * g.in + col];
          else if (g.out == 2 * g.in) y += g.Xf[row * g.in + (col >= g.in ? col - g.in : col)];
          g.Tt[row * g.out + col] = th;
          g.Y[row * g.out + col] = y;
        } else {
          float v = c;
          if (g.out == g.in || g.out == 2 * g.in) {
            v += wo ? wo[col] : g.gY[row * g.out + col];
            if (g.out == 2 * g.in) v += wo ? wo[col + g.in] : g.gY[row * g.out + col + g.in];
          }
          g.gX[row * g.in + col] = v;
        }
      }
}

// FP32 layers: v_mfma_f32_16x16x4f32, K staged in steps of 16
template <int MODE>
__global__ void __launch_bounds__(256) k_fitmix32(MG g) {
  __shared__ float As[64][17];
  __shared__ float Bs[16][64];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  if (r0 >= g.type_start[g.ntypes]) return;
  const int t = rtype(g.type_start, g.ntypes, r0);
  const float *W = (const float *)(g.w + g.fo.w32[t][g.layer]);
  const float *bias = (const float *)(g.w + g.fo.b32[t][g.layer]);
  const float *wo = (MODE == MF_BWD && g.gY == nullptr) ? (const float *)(g.w + g.fo.w32[t][g.layer + 1]) : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  v4f acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int rr = e >> 4, kk = e & 15, k = k0 + kk;
      float v = 0.f;
      if (k < g.K) {
        const int64_t row = r0 + rr;
        if (MODE == MF_FWD) {
          v = g.Xf[row * g.K + k];
        } else {
          const float th = g.Tt[row * g.K + k];
          const float gy = wo ? wo[k] : g.gY[row * g.K + k];
          v = gy * (1.f - th * th);
        }
      }
      As[rr][kk] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int kk = e >> 6, cc = e & 63, k = k0 + kk, c = c0 + cc;
      float v = 0.f;
      if (k < g.K && c < g.N) v = (MODE == MF_FWD) ? W[(int64_t)k * g.N + c] : W[(int64_t)c * g.K + k];
      Bs[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      float af[2], bf[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) af[mi] = As[wm * 32 + mi * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) bf[ni] = Bs[ks + (lane >> 4)][wn * 32 + ni * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + r;
        const int col = c0 + wn * 32 + ni * 16 + (lane & 15);
        if (col >= g.N) continue;
        const float c = acc[mi][ni][r];
        if (MODE == MF_FWD) {
          const float th = ftanh(c + bias[col]);
          float y = th;
          if (g.out == g.in) y += g.Xf[row * g.in + col];
          else if (g.out == 2 * g.in) y += g.Xf[row * g.in + (col >= g.in ? col - g.in : col)];
          g.Tt[row * g.out + col] = th;
          g.Y[row * g.out + col] = y;
        } else {
          float v = c;
          if (g.out == g.in || g.out == 2 * g.in) {
            v += wo ? wo[col] : g.gY[row * g.out + col];
            if (g.out == 2 * g.in) v += wo ? wo[col + g.in] : g.gY[row * g.out + col + g.in];
          }
          g.gX[row * g.in + col] = v;
        }
      }
}

__global__ void __launch_bounds__(256) k_fitmix_out(const int32_t *type_start, int ntypes, const int32_t *atom_of_pos,
                                                    const unsigned char *w, FitMixOffsets fo, int L, int width,
                                                    const float *Y, int64_t rows_cap, double *eatom) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_cap || row >= type_start[ntypes]) return;
  const int atom = atom_of_pos[row];
  if (atom < 0) return;
  const int t = rtype(type_start, ntypes, row);
  const float *wv = (const float *)(w + fo.w32[t][L]);
  float s = 0.f;
  for (int o = lane; o < width; o += 64) s += Y[row * width + o] * wv[o];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) eatom[atom] = (double)s + (double)((const float *)(w + fo.b32[t][L]))[0];
}

template <int P>
static void run(hipStream_t s, const FitMixArgs &a, int pass) {
  const Dims &d = a.d;
  const int L = d.n_fit;
  const unsigned gm = (unsigned)((a.rows + 63) / 64);
  for (int l = 0; l < L && pass == 1; ++l) {
    MG g{};
    g.layer = l;
    g.in = d.fw[l];
    g.out = d.fw[l + 1];
    g.K = g.in;
    g.N = g.out;
    g.ntypes = d.ntypes;
    g.type_start = a.type_start;
    g.w = a.w;
    g.fo = a.fo;
    g.Xf = (l == 0) ? a.X0 : a.Y[l];
    g.Tt = a.Tt[l + 1];
    g.Y = a.Y[l + 1];
    dim3 grid(gm, (unsigned)((g.N + 63) / 64));
    if (l < a.n16) hipLaunchKernelGGL((k_fitmix16<P, MF_FWD>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_fitmix32<MF_FWD>), grid, dim3(256), 0, s, g);
  }
  if (pass == 1)
    hipLaunchKernelGGL(k_fitmix_out, dim3((unsigned)((a.rows + 3) / 4)), dim3(256), 0, s, a.type_start, d.ntypes,
                       a.atom_of_pos, a.w, a.fo, L, d.fw[L], a.Y[L], a.rows, a.eatom);
  for (int l = L - 1; l >= 0 && pass == 2; --l) {
    MG g{};
    g.layer = l;
    g.in = d.fw[l];
    g.out = d.fw[l + 1];
    g.K = g.out;
    g.N = g.in;
    g.ntypes = d.ntypes;
    g.type_start = a.type_start;
    g.w = a.w;
    g.fo = a.fo;
    g.Tt = a.Tt[l + 1];
    g.gY = (l == L - 1) ? nullptr : a.G[l + 1];
    g.gX = a.G[l];
    dim3 grid(gm, (unsigned)((g.N + 63) / 64));
    if (l < a.n16) hipLaunchKernelGGL((k_fitmix16<P, MF_BWD>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_fitmix32<MF_BWD>), grid, dim3(256), 0, s, g);
  }
}

void launch_fit_mix(hipStream_t s, const FitMixArgs &a, int pass) {
  if (a.prec == 0) run<0>(s, a, pass);
  else run<1>(s, a, pass);
}

}  // namespace dpk
