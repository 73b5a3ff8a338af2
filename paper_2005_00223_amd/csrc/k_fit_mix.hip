// Mixed-precision fitting net (Fig. 1(d,g); Section V-B "Mixed-precision
// computation"), fused per tile of 16 type-sorted rows (one wave):
//
//   forward   D = T T_<^T is formed on the fly from T (M1 x 4 per atom) as
//             the B operand of the first layer, so D never reaches HBM; the
//             hidden layers chain in registers; E_i = Y w_out + b_out.
//   backward  from the stored tanh outputs: dE/dY through the hidden
//             layers, then dE/dD = W_0 dz_0 one 16-feature tile (one row a
//             of D) at a time, contracted at once with T into
//             dE/dT[a][c] = sum_b dD[a][b] T[b][c] + [a < M2] sum_a' dD[a'][a] T[a'][c],
//             so dD never reaches HBM either; dE/dT (times 1/Nc) is what the
//             embedding backward consumes.
//
// Layout.  Every layer is computed transposed (Y^T = W^T X^T, rows of the
// tile as the MFMA N dimension) with v_mfma_f32_16x16x32_{f16,bf16}.  The
// f32 output leaves lane (g = l/16, n = l%16) with features 16 mt + 4 g + r
// of row n in register r of output tile mt.  The next layer's k-step kk takes
// in lane group g the features 16 (2 kk + v/4) + 4 g + v%4 (v = 0..7), which
// are exactly the registers of output tiles 2 kk and 2 kk + 1, so activations
// never leave registers; the host stores every weight operand in that
// permuted K order, lane by lane (16 contiguous bytes per lane).  In the
// first layer, k-step kk covers D[a][b] with a = 2 kk + g/2 and
// b = 8 (g%2) + v.
//
// Precision.  Activations enter every product as hi + lo 16-bit halves
// (about 22 bits); the weights of the layers below `nsplit` are rounded to
// 16 bits (the paper's MIX scheme), the later hidden layers carry hi + lo
// weights as well (three products), tanh and all sums are FP32, E_i is
// converted to FP64 for the reduction.
#include <cstring>
#include <vector>

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

template <int P>
struct FSplit {
  typename FT<P>::v8 hi, lo;
};

// hi/lo halves of eight FP32 values x[0..3], y[0..3]
template <int P>
__device__ inline FSplit<P> fsplit(const float (&x)[4], const float (&y)[4]) {
  typedef typename FT<P>::e E;
  FSplit<P> s;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const E a = (E)x[v], b = (E)y[v];
    s.hi[v] = a;
    s.hi[v + 4] = b;
    s.lo[v] = (E)(x[v] - (float)a);
    s.lo[v + 4] = (E)(y[v] - (float)b);
  }
  return s;
}

template <>
__device__ inline FSplit<0> fsplit<0>(const float (&x)[4], const float (&y)[4]) {
  FSplit<0> s;
  split8_f16(x, y, s.hi, s.lo);
  return s;
}

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

constexpr int FIT_WAVES = 8;
constexpr int FIT_NT = 1;                           // 16-row tiles per wave
constexpr int FIT_ROWS = 16 * FIT_NT * FIT_WAVES;   // rows per workgroup
constexpr int FIT_MT = 15;                          // hidden width 240 = 15 output tiles
constexpr int FIT_KSH = (FIT_MT + 1) / 2;           // k-steps of a hidden layer
constexpr int STAGE_BYTES = 60 * 1024;              // one half of the double-buffered operand stage
constexpr int F0_CK = 4;                            // layer-0 k-steps per staged chunk (forward)
constexpr int FH_CK = 2;                            // hidden-layer k-steps per chunk (hi, then lo)
constexpr int F0_CA = 7;                            // rows of D per staged chunk (backward)
constexpr int FH_NC = FIT_KSH / FH_CK;              // chunks per hidden layer
static_assert(FIT_ROWS == ROW_TILE, "a workgroup's rows must share one type");
static_assert(F0_CK * FIT_MT * 1024 <= STAGE_BYTES && 2 * FH_CK * FIT_MT * 1024 <= STAGE_BYTES &&
                  F0_CA * FIT_KSH * 1024 <= STAGE_BYTES && FIT_KSH % FH_CK == 0,
              "staged chunks must fit one half of the stage");

// One 1 KB operand block (64 lanes x 16 B) from global memory straight into
// LDS (global_load_lds_dwordx4, no registers); lds must be wave-uniform.
__device__ inline void dma_1k(const unsigned char *src, unsigned char *lds, int lane) {
  __builtin_amdgcn_global_load_lds((const void *)(src + 16 * lane), (__attribute__((address_space(3))) void *)lds, 16,
                                   0, 0);
}

// the waves of the block stage blocks [b0, b0 + nb) of an image into buf
__device__ inline void dma_blocks(const unsigned char *img, int64_t b0, int nb, unsigned char *buf, int wv, int lane) {
  for (int b = wv; b < nb; b += FIT_WAVES) dma_1k(img + (b0 + b) * 1024, buf + b * 1024, lane);
}

__device__ inline void dma_wait_all() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// per row tile in tbuf: [layer][mt][lane][4] floats
template <int MT>
__device__ inline float *tile_t(float *tbuf, int64_t tile, int nl, int l, int mt) {
  return tbuf + (((tile * nl + l) * MT + mt) * 64) * 4;
}

// Staged chunk gc of the forward: layer-0 chunks (F0_CK k-steps of the
// [kk][mt] image), then FH_NC chunks per hidden layer (FH_CK k-steps of the
// hi image, followed by the same k-steps of the lo image when the layer
// carries one).
__device__ inline void fwd_issue(const FitMixArgs &a, int t, int gc, int n0c, unsigned char *buf, int wv, int lane) {
  if (gc < n0c) {
    const int KS0 = a.d.M1 / 2, k0 = gc * F0_CK, nk = KS0 - k0 < F0_CK ? KS0 - k0 : F0_CK;
    dma_blocks(a.w + a.fo.a0f[t], (int64_t)k0 * FIT_MT, nk * FIT_MT, buf, wv, lane);
  } else {
    const int h = gc - n0c, l = 1 + h / FH_NC, c = h % FH_NC;
    dma_blocks(a.w + a.fo.ahf[t][l], (int64_t)c * FH_CK * FIT_MT, FH_CK * FIT_MT, buf, wv, lane);
    if (l >= a.nsplit)
      dma_blocks(a.w + a.fo.ahf_lo[t][l], (int64_t)c * FH_CK * FIT_MT, FH_CK * FIT_MT, buf + FH_CK * FIT_MT * 1024,
                 wv, lane);
  }
}

// Staged chunk gc of the backward: FH_NC chunks per hidden layer from the
// last down to layer 1, then layer-0 chunks of F0_CA rows of D ([aa][kk]).
__device__ inline void bwd_issue(const FitMixArgs &a, int t, int gc, unsigned char *buf, int wv, int lane) {
  const int nh = (a.d.n_fit - 1) * FH_NC;
  if (gc < nh) {
    const int l = a.d.n_fit - 1 - gc / FH_NC, c = gc % FH_NC;
    dma_blocks(a.w + a.fo.ahb[t][l], (int64_t)c * FH_CK * FIT_MT, FH_CK * FIT_MT, buf, wv, lane);
    if (l >= a.nsplit)
      dma_blocks(a.w + a.fo.ahb_lo[t][l], (int64_t)c * FH_CK * FIT_MT, FH_CK * FIT_MT, buf + FH_CK * FIT_MT * 1024,
                 wv, lane);
  } else {
    const int M1 = a.d.M1, a0 = (gc - nh) * F0_CA, na = M1 - a0 < F0_CA ? M1 - a0 : F0_CA;
    dma_blocks(a.w + a.fo.a0b[t], (int64_t)a0 * FIT_KSH, na * FIT_KSH, buf, wv, lane);
  }
}

// One hidden layer over its FH_NC staged chunks: acc[nt][mt] += A X for the
// wave's tiles, X of k-step kk = the split halves xs[nt][kk] built by bx(nt,
// kk, x, y) on the fly; SPLIT adds the lo weights (three products).  Every
// chunk prefetches the next one of the sequence (issue) and ends with the
// block barrier.
template <int P, int MT, bool SPLIT, class Issue, class BX>
__device__ inline void hidden_layer(unsigned char (*stage)[STAGE_BYTES], int &gc, int nchunks, Issue issue, BX bx,
                                    v4f (&acc)[FIT_NT][MT], int lane) {
  typedef typename FT<P>::v8 V;
#pragma unroll
  for (int c = 0; c < FH_NC; ++c, ++gc) {
    if (gc + 1 < nchunks) issue(gc + 1, stage[(gc + 1) & 1]);
    const unsigned char *buf = stage[gc & 1];
#pragma unroll
    for (int q = 0; q < FH_CK; ++q) {
      const int kk = c * FH_CK + q;
      FSplit<P> B[FIT_NT];
#pragma unroll
      for (int nt = 0; nt < FIT_NT; ++nt) {
        float x[4], y[4];
        bx(nt, kk, x, y);
        B[nt] = fsplit<P>(x, y);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const V ah = *(const V *)(buf + (q * MT + mt) * 1024 + 16 * lane);
#pragma unroll
        for (int nt = 0; nt < FIT_NT; ++nt) {
          acc[nt][mt] = FT<P>::mma(ah, B[nt].hi, acc[nt][mt]);
          acc[nt][mt] = FT<P>::mma(ah, B[nt].lo, acc[nt][mt]);
        }
        if (SPLIT) {
          const V al = *(const V *)(buf + ((FH_CK + q) * MT + mt) * 1024 + 16 * lane);
#pragma unroll
          for (int nt = 0; nt < FIT_NT; ++nt) acc[nt][mt] = FT<P>::mma(al, B[nt].hi, acc[nt][mt]);
        }
      }
    }
    dma_wait_all();
  }
}

// Forward: one workgroup = FIT_ROWS rows of one type, one wave = FIT_NT
// tiles of 16 rows sharing every operand read from LDS.
template <int P, int MT>
__global__ void __launch_bounds__(64 * FIT_WAVES, 1) k_fit_fwd(FitMixArgs a) {
  typedef typename FT<P>::v8 V;
  constexpr int NT = FIT_NT;
  __shared__ __align__(16) unsigned char stage[2][STAGE_BYTES];
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, wv = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * FIT_ROWS;
  const int ntypes = a.d.ntypes;
  // a block's rows share one type (types are padded to FIT_ROWS rows) or lie
  // past the end: the exit is block-uniform, so the barriers below are safe
  if (r0 >= a.type_start[ntypes]) return;
  const int t = rtype(a.type_start, ntypes, r0);
  const int M1 = a.d.M1, NL = a.d.n_fit, KS0 = M1 / 2;
  const int64_t tile0 = r0 / 16 + (int64_t)wv * NT;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  // padding rows (ia < 0) read atom 0's T, scaled by 0 in Tb: every load is
  // unconditional, so none of them waits behind a branch (M1 >= 16)
  int ia[NT];
  const float4 *Ti[NT];
  float4 Tb[NT][8];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    ia[nt] = a.atom_of_pos[(tile0 + nt) * 16 + n];
    Ti[nt] = (const float4 *)(a.T32 + (int64_t)(ia[nt] < 0 ? 0 : ia[nt]) * M1 * 4);
    const float live = ia[nt] >= 0 ? 1.f : 0.f;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const float4 q = Ti[nt][8 * (g & 1) + v];
      Tb[nt][v] = make_float4(q.x * live, q.y * live, q.z * live, q.w * live);
    }
  }
  const unsigned char *W = a.w;
  const int n0c = (KS0 + F0_CK - 1) / F0_CK, nchunks = n0c + (NL - 1) * FH_NC;
  auto issue = [&](int c, unsigned char *buf) { fwd_issue(a, t, c, n0c, buf, wv, lane); };
  issue(0, stage[0]);
  v4f acc[NT][MT];
  {
    const float *b0 = (const float *)(W + a.fo.bias[t][0]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 b = *(const float4 *)(b0 + 16 * mt + 4 * g);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = v4f{b.x, b.y, b.z, b.w};
    }
  }
  // layer 0: K = M1*16 features of D = T T<^T, formed from T as the B operand
  float4 Ta[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) Ta[nt] = Ti[nt][g >> 1];
  dma_wait_all();
  int gc = 0;
  for (int c = 0; c < n0c; ++c, ++gc) {
    if (gc + 1 < nchunks) issue(gc + 1, stage[(gc + 1) & 1]);
    const unsigned char *buf = stage[gc & 1];
#pragma unroll
    for (int q = 0; q < F0_CK; ++q) {
      const int kk = c * F0_CK + q;
      if (kk < KS0) {
        FSplit<P> B[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const float4 ta = Ta[nt];
          float x[4], y[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            x[v] = ta.x * Tb[nt][v].x + ta.y * Tb[nt][v].y + ta.z * Tb[nt][v].z + ta.w * Tb[nt][v].w;
            y[v] = ta.x * Tb[nt][v + 4].x + ta.y * Tb[nt][v + 4].y + ta.z * Tb[nt][v + 4].z + ta.w * Tb[nt][v + 4].w;
          }
          B[nt] = fsplit<P>(x, y);
          // next k-step's row a of T, in flight during this one's products
          if (kk + 1 < KS0) Ta[nt] = Ti[nt][2 * (kk + 1) + (g >> 1)];
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const V av = *(const V *)(buf + (q * MT + mt) * 1024 + 16 * lane);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            acc[nt][mt] = FT<P>::mma(av, B[nt].hi, acc[nt][mt]);
            acc[nt][mt] = FT<P>::mma(av, B[nt].lo, acc[nt][mt]);
          }
        }
      }
    }
    dma_wait_all();
  }
  float Y[NT][MT][4];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float th[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        th[r] = ftanh(acc[nt][mt][r]);
        Y[nt][mt][r] = th[r];
      }
      *(float4 *)(tile_t<MT>(a.tbuf, tile0 + nt, NL, 0, mt) + 4 * lane) = make_float4(th[0], th[1], th[2], th[3]);
    }
  // hidden layers 1 .. NL-1 (identity skip): the B operand of k-step kk is
  // made of output tiles 2kk and 2kk+1 of the layer below
  auto bx = [&](int nt, int kk, float (&x)[4], float (&y)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      x[v] = Y[nt][2 * kk][v];
      y[v] = (2 * kk + 1 < MT) ? Y[nt][(2 * kk + 1 < MT) ? 2 * kk + 1 : 0][v] : 0.f;
    }
  };
  for (int l = 1; l < NL; ++l) {
    const float *bl = (const float *)(W + a.fo.bias[t][l]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 b = *(const float4 *)(bl + 16 * mt + 4 * g);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt][mt] = v4f{b.x, b.y, b.z, b.w};
    }
    if (l >= a.nsplit) hidden_layer<P, MT, true>(stage, gc, nchunks, issue, bx, acc, lane);
    else hidden_layer<P, MT, false>(stage, gc, nchunks, issue, bx, acc, lane);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float th[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          th[r] = ftanh(acc[nt][mt][r]);
          Y[nt][mt][r] += th[r];
        }
        *(float4 *)(tile_t<MT>(a.tbuf, tile0 + nt, NL, l, mt) + 4 * lane) = make_float4(th[0], th[1], th[2], th[3]);
      }
  }
  // output layer
  const float *wo = (const float *)(W + a.fo.wout[t]);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    float e = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 w4 = *(const float4 *)(wo + 16 * mt + 4 * g);
      e += Y[nt][mt][0] * w4.x + Y[nt][mt][1] * w4.y + Y[nt][mt][2] * w4.z + Y[nt][mt][3] * w4.w;
    }
    e += __shfl_xor(e, 16);
    e += __shfl_xor(e, 32);
    if (g == 0 && ia[nt] >= 0) a.eatom[ia[nt]] = (double)e + (double)wo[256];
  }
}

template <int P, int MT>
__global__ void __launch_bounds__(64 * FIT_WAVES, 1) k_fit_bwd(FitMixArgs a) {
  typedef typename FT<P>::v8 V;
  constexpr int NT = FIT_NT, KSH = (MT + 1) / 2;
  __shared__ float4 sh[FIT_WAVES][NT][16][16];  // per tile: sum_b dD[a][b] T[b] for a < 16
  __shared__ __align__(16) unsigned char stage[2][STAGE_BYTES];
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, wv = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * FIT_ROWS;
  const int ntypes = a.d.ntypes;
  if (r0 >= a.type_start[ntypes]) return;  // block-uniform
  const int t = rtype(a.type_start, ntypes, r0);
  const int M1 = a.d.M1, NL = a.d.n_fit;
  const int64_t tile0 = r0 / 16 + (int64_t)wv * NT;
  const unsigned char *W = a.w;
  int ia[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) ia[nt] = a.atom_of_pos[(tile0 + nt) * 16 + n];
  const int n0c = (M1 + F0_CA - 1) / F0_CA, nchunks = (NL - 1) * FH_NC + n0c;
  auto issue = [&](int c, unsigned char *buf) { bwd_issue(a, t, c, buf, wv, lane); };
  issue(0, stage[0]);
  // dE/dY of the last hidden layer = w_out
  float dY[NT][MT][4];
  {
    const float *wo = (const float *)(W + a.fo.wout[t]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 w4 = *(const float4 *)(wo + 16 * mt + 4 * g);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        dY[nt][mt][0] = w4.x;
        dY[nt][mt][1] = w4.y;
        dY[nt][mt][2] = w4.z;
        dY[nt][mt][3] = w4.w;
      }
    }
  }
  dma_wait_all();
  int gc = 0;
  // hidden layers NL-1 .. 1: dY_{l-1} = W_l dz_l + dY_l, dz_l = dY_l (1 - t_l^2);
  // the tanh outputs of k-step kk (tiles 2kk, 2kk+1) are loaded two k-steps ahead
  for (int l = NL - 1; l >= 1; --l) {
    float4 tp[2][NT][2];
    auto tload = [&](int kk, float4 (&dst)[NT][2]) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        dst[nt][0] = *(const float4 *)(tile_t<MT>(a.tbuf, tile0 + nt, NL, l, 2 * kk) + 4 * lane);
        const int m1 = (2 * kk + 1 < MT) ? 2 * kk + 1 : 2 * kk;
        dst[nt][1] = *(const float4 *)(tile_t<MT>(a.tbuf, tile0 + nt, NL, l, m1) + 4 * lane);
      }
    };
    tload(0, tp[0]);
    tload(1, tp[1]);
    v4f acc[NT][MT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = v4f{0.f, 0.f, 0.f, 0.f};
    auto bx = [&](int nt, int kk, float (&x)[4], float (&y)[4]) {
      const float4 t0 = tp[kk & 1][nt][0], t1 = tp[kk & 1][nt][1];
      const float tv0[4] = {t0.x, t0.y, t0.z, t0.w}, tv1[4] = {t1.x, t1.y, t1.z, t1.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x[v] = dY[nt][2 * kk][v] * (1.f - tv0[v] * tv0[v]);
        y[v] = (2 * kk + 1 < MT) ? dY[nt][(2 * kk + 1 < MT) ? 2 * kk + 1 : 0][v] * (1.f - tv1[v] * tv1[v]) : 0.f;
      }
      if (nt == NT - 1 && kk + 2 < KSH) tload(kk + 2, tp[kk & 1]);
    };
    if (l >= a.nsplit) hidden_layer<P, MT, true>(stage, gc, nchunks, issue, bx, acc, lane);
    else hidden_layer<P, MT, false>(stage, gc, nchunks, issue, bx, acc, lane);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dY[nt][mt][r] += acc[nt][mt][r];
  }
  // dz_0 as the B operands of the first layer's backward
  FSplit<P> Bz[NT][KSH];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int kk = 0; kk < KSH; ++kk) {
      float x[4], y[4];
      const float4 t0 = *(const float4 *)(tile_t<MT>(a.tbuf, tile0 + nt, NL, 0, 2 * kk) + 4 * lane);
      const float tv0[4] = {t0.x, t0.y, t0.z, t0.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) x[v] = dY[nt][2 * kk][v] * (1.f - tv0[v] * tv0[v]);
      if (2 * kk + 1 < MT) {
        const int m1 = (2 * kk + 1 < MT) ? 2 * kk + 1 : 0;
        const float4 t1 = *(const float4 *)(tile_t<MT>(a.tbuf, tile0 + nt, NL, 0, m1) + 4 * lane);
        const float tv1[4] = {t1.x, t1.y, t1.z, t1.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] = dY[nt][m1][v] * (1.f - tv1[v] * tv1[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] = 0.f;
      }
      Bz[nt][kk] = fsplit<P>(x, y);
    }
  // dD one row a of D (16 features b) at a time, contracted with T:
  //   dE/dT[a][c] = sum_b dD[a][b] T[b][c] + [a < M2] sum_a' dD[a'][a] T[a'][c]
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 *Ti[NT];
  float4 *dTi[NT];
  float4 Tq[NT][4], Ta[NT];
  float dT2[NT][4][4];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    Ti[nt] = (const float4 *)(a.T32 + (int64_t)(ia[nt] < 0 ? 0 : ia[nt]) * M1 * 4);
    dTi[nt] = (float4 *)(a.dT32 + (int64_t)(ia[nt] < 0 ? 0 : ia[nt]) * M1 * 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) Tq[nt][r] = Ti[nt][4 * g + r];  // padding rows: results never stored
    Ta[nt] = Ti[nt][0];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) dT2[nt][r][c] = 0.f;
  }
  const float s = a.inv_nc;
  for (int ch = 0; ch < n0c; ++ch, ++gc) {
    if (gc + 1 < nchunks) issue(gc + 1, stage[(gc + 1) & 1]);
    const unsigned char *buf = stage[gc & 1];
    for (int q = 0; q < F0_CA; ++q) {
      const int aa = ch * F0_CA + q;
      if (aa >= M1) break;
      v4f cc[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) cc[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < KSH; ++kk) {
        const V av = *(const V *)(buf + (q * KSH + kk) * 1024 + 16 * lane);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          cc[nt] = FT<P>::mma(av, Bz[nt][kk].hi, cc[nt]);
          cc[nt] = FT<P>::mma(av, Bz[nt][kk].lo, cc[nt]);
        }
      }
      // cc[nt][r] = dE/dD[row n][a = aa][b = 4 g + r]
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const v4f c = cc[nt];
        const float4 ta = Ta[nt];
        if (aa + 1 < M1) Ta[nt] = Ti[nt][aa + 1];
        float4 pc;
        pc.x = c[0] * Tq[nt][0].x + c[1] * Tq[nt][1].x + c[2] * Tq[nt][2].x + c[3] * Tq[nt][3].x;
        pc.y = c[0] * Tq[nt][0].y + c[1] * Tq[nt][1].y + c[2] * Tq[nt][2].y + c[3] * Tq[nt][3].y;
        pc.z = c[0] * Tq[nt][0].z + c[1] * Tq[nt][1].z + c[2] * Tq[nt][2].z + c[3] * Tq[nt][3].z;
        pc.w = c[0] * Tq[nt][0].w + c[1] * Tq[nt][1].w + c[2] * Tq[nt][2].w + c[3] * Tq[nt][3].w;
        pc.x += __shfl_xor(pc.x, 16);
        pc.y += __shfl_xor(pc.y, 16);
        pc.z += __shfl_xor(pc.z, 16);
        pc.w += __shfl_xor(pc.w, 16);
        pc.x += __shfl_xor(pc.x, 32);
        pc.y += __shfl_xor(pc.y, 32);
        pc.z += __shfl_xor(pc.z, 32);
        pc.w += __shfl_xor(pc.w, 32);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          dT2[nt][r][0] += c[r] * ta.x;
          dT2[nt][r][1] += c[r] * ta.y;
          dT2[nt][r][2] += c[r] * ta.z;
          dT2[nt][r][3] += c[r] * ta.w;
        }
        if (g == 0) {
          if (aa < 16) sh[wv][nt][n][aa] = pc;
          else if (ia[nt] >= 0) dTi[nt][aa] = make_float4(pc.x * s, pc.y * s, pc.z * s, pc.w * s);
        }
      }
    }
    dma_wait_all();
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    if (ia[nt] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = 4 * g + r;
      if (b < M1) {
        const float4 q = sh[wv][nt][n][b];
        dTi[nt][b] = make_float4((q.x + dT2[nt][r][0]) * s, (q.y + dT2[nt][r][1]) * s, (q.z + dT2[nt][r][2]) * s,
                                 (q.w + dT2[nt][r][3]) * s);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
bool fit_mix_supported(const Dims &d, const char **why) {
  const int H = d.fw[1];
  for (int l = 1; l <= d.n_fit; ++l)
    if (d.fw[l] != H) return *why = "mixed fitting net needs equal hidden widths", false;
  if (H != 16 * FIT_MT) return *why = "mixed fitting net is built for hidden width 240", false;
  if (d.M2 != 16) return *why = "mixed fitting net needs M2 = 16", false;
  if (d.M1 % 2 != 0 || d.M1 < 16 || d.M1 > 2048) return *why = "mixed fitting net needs an even M1 in 16..2048", false;
  if (d.n_fit < 1 || d.n_fit > MAXF) return *why = "mixed fitting net needs 1..4 hidden layers", false;
  return true;
}

static inline uint16_t bits16(double v, int prec) {
  const float f = (float)v;
  if (prec == 0) {
    _Float16 h = (_Float16)f;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
  }
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static inline double val16(uint16_t u, int prec) {
  if (prec == 0) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return (double)(float)h;
  }
  const uint32_t w = (uint32_t)u << 16;
  float f;
  std::memcpy(&f, &w, 4);
  return (double)f;
}

// 16-bit operand image: nt tiles x ks k-steps x 64 lanes x 8, element value
// from fn(tile, kk, lane, v) (lo = true: the rounding remainder)
template <class F>
static int64_t put_image(std::vector<unsigned char> &buf, int nt, int ks, int prec, bool lo, F fn) {
  buf.resize((buf.size() + 255) / 256 * 256, 0);
  const int64_t off = (int64_t)buf.size();
  buf.resize(buf.size() + (size_t)nt * ks * 64 * 8 * 2, 0);
  uint16_t *p = (uint16_t *)(buf.data() + off);
  for (int tl = 0; tl < nt; ++tl)
    for (int kk = 0; kk < ks; ++kk)
      for (int lane = 0; lane < 64; ++lane)
        for (int v = 0; v < 8; ++v) {
          const double x = fn(tl, kk, lane, v);
          const uint16_t h = bits16(x, prec);
          p[(((size_t)tl * ks + kk) * 64 + lane) * 8 + v] = lo ? bits16(x - val16(h, prec), prec) : h;
        }
  return off;
}

static int64_t put_f32(std::vector<unsigned char> &buf, const std::vector<float> &v) {
  buf.resize((buf.size() + 255) / 256 * 256, 0);
  const int64_t off = (int64_t)buf.size();
  buf.resize(buf.size() + 4 * v.size(), 0);
  std::memcpy(buf.data() + off, v.data(), 4 * v.size());
  return off;
}

void fit_mix_pack(const Dims &d, int prec, int nsplit, const double *const *W, const double *const *b,
                  std::vector<unsigned char> &buf, FitMixOffsets &fo) {
  const int H = d.fw[1], M1 = d.M1, NL = d.n_fit, MT = FIT_MT, KSH = (MT + 1) / 2, KS0 = M1 / 2;
  auto kslot = [](int kk, int g, int v) { return 16 * (2 * kk + v / 4) + 4 * g + (v % 4); };
  fo = FitMixOffsets{};
  for (int t = 0; t < d.ntypes; ++t) {
    const double *const *Wt = W + (size_t)t * (NL + 1);
    const double *const *bt = b + (size_t)t * (NL + 1);
    const int K0 = d.fw[0];  // M1 * 16
    // layer 0 forward, blocks in [kk][mt] order: A[o][k] = W0[k][o], k of
    // slot (kk, g, v) = (2kk + g/2)*16 + 8(g%2) + v
    fo.a0f[t] = put_image(buf, KS0, MT, prec, false, [&](int kk, int mt, int lane, int v) {
      const int g = lane >> 4, o = 16 * mt + (lane & 15);
      const int k = (2 * kk + (g >> 1)) * 16 + 8 * (g & 1) + v;
      return (o < H && k < K0) ? Wt[0][(size_t)k * H + o] : 0.0;
    });
    // layer 0 backward: A[k][o] = W0[k][o], k = 16 a + lane%16, o = kslot
    fo.a0b[t] = put_image(buf, M1, KSH, prec, false, [&](int aa, int kk, int lane, int v) {
      const int k = 16 * aa + (lane & 15), o = kslot(kk, lane >> 4, v);
      return (o < H && k < K0) ? Wt[0][(size_t)k * H + o] : 0.0;
    });
    for (int l = 1; l < NL; ++l) {
      auto fwd = [&](int mt, int kk, int lane, int v) {
        const int o = 16 * mt + (lane & 15), k = kslot(kk, lane >> 4, v);
        return (o < H && k < H) ? Wt[l][(size_t)k * H + o] : 0.0;
      };
      auto bwd = [&](int mt, int kk, int lane, int v) {
        const int k = 16 * mt + (lane & 15), o = kslot(kk, lane >> 4, v);
        return (o < H && k < H) ? Wt[l][(size_t)k * H + o] : 0.0;
      };
      // blocks in [kk][mt] order: a staged chunk of k-steps is contiguous
      auto fwd_km = [&](int kk, int mt, int lane, int v) { return fwd(mt, kk, lane, v); };
      auto bwd_km = [&](int kk, int mt, int lane, int v) { return bwd(mt, kk, lane, v); };
      fo.ahf[t][l] = put_image(buf, KSH, MT, prec, false, fwd_km);
      fo.ahb[t][l] = put_image(buf, KSH, MT, prec, false, bwd_km);
      if (l >= nsplit) {
        fo.ahf_lo[t][l] = put_image(buf, KSH, MT, prec, true, fwd_km);
        fo.ahb_lo[t][l] = put_image(buf, KSH, MT, prec, true, bwd_km);
      } else {
        fo.ahf_lo[t][l] = fo.ahf[t][l];
        fo.ahb_lo[t][l] = fo.ahb[t][l];
      }
    }
    for (int l = 0; l < NL; ++l) {
      std::vector<float> bias(256, 0.f);
      for (int o = 0; o < H; ++o) bias[o] = (float)bt[l][o];
      fo.bias[t][l] = put_f32(buf, bias);
    }
    std::vector<float> wo(260, 0.f);
    for (int f = 0; f < H; ++f) wo[f] = (float)Wt[NL][f];
    wo[256] = (float)bt[NL][0];
    fo.wout[t] = put_f32(buf, wo);
  }
  buf.resize((buf.size() + 255) / 256 * 256, 0);
}

size_t fit_mix_tbuf_floats(const Dims &d, int64_t rows) {
  return (size_t)((rows + 15) / 16) * d.n_fit * FIT_MT * 256;
}

void launch_fit_mix(hipStream_t s, const FitMixArgs &a, int pass) {
  const unsigned grid = (unsigned)((a.rows + FIT_ROWS - 1) / FIT_ROWS);
  if (grid == 0) return;
  if (pass == 1) {
    if (a.prec == 0) hipLaunchKernelGGL((k_fit_fwd<0, FIT_MT>), dim3(grid), dim3(64 * FIT_WAVES), 0, s, a);
    else hipLaunchKernelGGL((k_fit_fwd<1, FIT_MT>), dim3(grid), dim3(64 * FIT_WAVES), 0, s, a);
  } else {
    if (a.prec == 0) hipLaunchKernelGGL((k_fit_bwd<0, FIT_MT>), dim3(grid), dim3(64 * FIT_WAVES), 0, s, a);
    else hipLaunchKernelGGL((k_fit_bwd<1, FIT_MT>), dim3(grid), dim3(64 * FIT_WAVES), 0, s, a);
  }
}

}  // namespace dpk
