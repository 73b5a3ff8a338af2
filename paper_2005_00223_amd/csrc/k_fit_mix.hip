// Mixed-precision fitting net (Fig. 1(d,g); Section V-A "Mixed-precision
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

constexpr int FIT_WAVES = 4;
constexpr int F0_CK = 2;  // first-layer k-steps per staged chunk (forward)
constexpr int F0_CA = 4;  // rows of D per staged chunk (backward)

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

template <int P, int MT>
__global__ void __launch_bounds__(64 * FIT_WAVES, 2) k_fit_fwd(FitMixArgs a) {
  typedef typename FT<P>::v8 V;
  constexpr int KSH = (MT + 1) / 2;
  __shared__ __align__(16) unsigned char stage[2][F0_CK * MT * 1024];
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * FIT_WAVES + wv;
  const int64_t p0 = tile * 16;
  const int ntypes = a.d.ntypes;
  // a block's 64 rows share one type (types are padded to 64 rows) or lie
  // past the end: the exit is block-uniform, so the barriers below are safe
  if ((int64_t)blockIdx.x * 16 * FIT_WAVES >= a.type_start[ntypes]) return;
  const int t = rtype(a.type_start, ntypes, p0);
  const int i = a.atom_of_pos[p0 + n];
  const int M1 = a.d.M1, NL = a.d.n_fit;
  const float4 *Ti = (const float4 *)(a.T32 + (int64_t)(i < 0 ? 0 : i) * M1 * 4);
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 Tb[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) Tb[v] = i >= 0 ? Ti[8 * (g & 1) + v] : z4;
  const unsigned char *W = a.w;
  v4f acc[MT];
  {
    const float *b0 = (const float *)(W + a.fo.bias[t][0]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 b = *(const float4 *)(b0 + 16 * mt + 4 * g);
      acc[mt] = v4f{b.x, b.y, b.z, b.w};
    }
  }
  // layer 0: K = M1*16 features of D, formed from T.  The A operands
  // ([kk][mt] blocks of 1 KB) stream through LDS in chunks of F0_CK k-steps,
  // the next chunk loading while this one is used.
  const unsigned char *A0 = W + a.fo.a0f[t];
  const int KS0 = M1 / 2;
  const int nch = (KS0 + F0_CK - 1) / F0_CK;
  dma_blocks(A0, 0, (KS0 < F0_CK ? KS0 : F0_CK) * MT, stage[0], wv, lane);
  dma_wait_all();
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) {
      const int k1 = (c + 1) * F0_CK, nk = (KS0 - k1 < F0_CK) ? KS0 - k1 : F0_CK;
      dma_blocks(A0, (int64_t)k1 * MT, nk * MT, stage[(c + 1) & 1], wv, lane);
    }
    const unsigned char *buf = stage[c & 1];
#pragma unroll
    for (int q = 0; q < F0_CK; ++q) {
      const int kk = c * F0_CK + q;
      if (kk < KS0) {
        const float4 Ta = i >= 0 ? Ti[2 * kk + (g >> 1)] : z4;
        float x[4], y[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          x[v] = Ta.x * Tb[v].x + Ta.y * Tb[v].y + Ta.z * Tb[v].z + Ta.w * Tb[v].w;
          y[v] = Ta.x * Tb[v + 4].x + Ta.y * Tb[v + 4].y + Ta.z * Tb[v + 4].z + Ta.w * Tb[v + 4].w;
        }
        const FSplit<P> B = fsplit<P>(x, y);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const V av = *(const V *)(buf + (q * MT + mt) * 1024 + 16 * lane);
          acc[mt] = FT<P>::mma(av, B.hi, acc[mt]);
          acc[mt] = FT<P>::mma(av, B.lo, acc[mt]);
        }
      }
    }
    dma_wait_all();
  }
  float Y[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    float th[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      th[r] = ftanh(acc[mt][r]);
      Y[mt][r] = th[r];
    }
    *(float4 *)(tile_t<MT>(a.tbuf, tile, NL, 0, mt) + 4 * lane) = make_float4(th[0], th[1], th[2], th[3]);
  }
  // hidden layers 1 .. NL-1 (identity skip)
  for (int l = 1; l < NL; ++l) {
    const float *bl = (const float *)(W + a.fo.bias[t][l]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 b = *(const float4 *)(bl + 16 * mt + 4 * g);
      acc[mt] = v4f{b.x, b.y, b.z, b.w};
    }
    const V *Ah = (const V *)(W + a.fo.ahf[t][l]);
    const bool split = l >= a.nsplit;
    const V *Al = (const V *)(W + a.fo.ahf_lo[t][l]);
#pragma unroll
    for (int kk = 0; kk < KSH; ++kk) {
      float x[4], y[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x[v] = Y[2 * kk][v];
        y[v] = (2 * kk + 1 < MT) ? Y[(2 * kk + 1 < MT) ? 2 * kk + 1 : 0][v] : 0.f;
      }
      const FSplit<P> B = fsplit<P>(x, y);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const V ah = Ah[(mt * KSH + kk) * 64 + lane];
        acc[mt] = FT<P>::mma(ah, B.hi, acc[mt]);
        acc[mt] = FT<P>::mma(ah, B.lo, acc[mt]);
        if (split) {
          const V al = Al[(mt * KSH + kk) * 64 + lane];
          acc[mt] = FT<P>::mma(al, B.hi, acc[mt]);
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float th[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        th[r] = ftanh(acc[mt][r]);
        Y[mt][r] += th[r];
      }
      *(float4 *)(tile_t<MT>(a.tbuf, tile, NL, l, mt) + 4 * lane) = make_float4(th[0], th[1], th[2], th[3]);
    }
  }
  // output layer
  const float *wo = (const float *)(W + a.fo.wout[t]);
  float e = 0.f;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const float4 w4 = *(const float4 *)(wo + 16 * mt + 4 * g);
    e += Y[mt][0] * w4.x + Y[mt][1] * w4.y + Y[mt][2] * w4.z + Y[mt][3] * w4.w;
  }
  e += __shfl_xor(e, 16);
  e += __shfl_xor(e, 32);
  if (g == 0 && i >= 0) a.eatom[i] = (double)e + (double)wo[256];
}

template <int P, int MT>
__global__ void __launch_bounds__(64 * FIT_WAVES, 2) k_fit_bwd(FitMixArgs a) {
  typedef typename FT<P>::v8 V;
  constexpr int KSH = (MT + 1) / 2;
  __shared__ float4 sh[FIT_WAVES][16][16];  // per wave: sum_b dD[a][b] T[b] for a < 16
  __shared__ __align__(16) unsigned char stage[2][F0_CA * KSH * 1024];
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * FIT_WAVES + wv;
  const int64_t p0 = tile * 16;
  const int ntypes = a.d.ntypes;
  if ((int64_t)blockIdx.x * 16 * FIT_WAVES >= a.type_start[ntypes]) return;  // block-uniform
  const int t = rtype(a.type_start, ntypes, p0);
  const int i = a.atom_of_pos[p0 + n];
  const int M1 = a.d.M1, NL = a.d.n_fit;
  const unsigned char *W = a.w;
  // dE/dY of the last hidden layer = w_out
  float dY[MT][4];
  {
    const float *wo = (const float *)(W + a.fo.wout[t]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const float4 w4 = *(const float4 *)(wo + 16 * mt + 4 * g);
      dY[mt][0] = w4.x;
      dY[mt][1] = w4.y;
      dY[mt][2] = w4.z;
      dY[mt][3] = w4.w;
    }
  }
  // hidden layers NL-1 .. 1: dY_{l-1} = W_l dz_l + dY_l, dz_l = dY_l (1 - t_l^2)
  for (int l = NL - 1; l >= 1; --l) {
    const V *Ah = (const V *)(W + a.fo.ahb[t][l]);
    const bool split = l >= a.nsplit;
    const V *Al = (const V *)(W + a.fo.ahb_lo[t][l]);
    v4f acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < KSH; ++kk) {
      float x[4], y[4];
      {
        const float4 t0 = *(const float4 *)(tile_t<MT>(a.tbuf, tile, NL, l, 2 * kk) + 4 * lane);
        const float tv[4] = {t0.x, t0.y, t0.z, t0.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = dY[2 * kk][v] * (1.f - tv[v] * tv[v]);
      }
      if (2 * kk + 1 < MT) {
        const int m1 = (2 * kk + 1 < MT) ? 2 * kk + 1 : 0;
        const float4 t1 = *(const float4 *)(tile_t<MT>(a.tbuf, tile, NL, l, m1) + 4 * lane);
        const float tv[4] = {t1.x, t1.y, t1.z, t1.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] = dY[m1][v] * (1.f - tv[v] * tv[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] = 0.f;
      }
      const FSplit<P> B = fsplit<P>(x, y);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const V ah = Ah[(mt * KSH + kk) * 64 + lane];
        acc[mt] = FT<P>::mma(ah, B.hi, acc[mt]);
        acc[mt] = FT<P>::mma(ah, B.lo, acc[mt]);
        if (split) {
          const V al = Al[(mt * KSH + kk) * 64 + lane];
          acc[mt] = FT<P>::mma(al, B.hi, acc[mt]);
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) dY[mt][r] += acc[mt][r];
  }
  // dz_0 as the B operands of the first layer's backward
  FSplit<P> Bz[KSH];
#pragma unroll
  for (int kk = 0; kk < KSH; ++kk) {
    float x[4], y[4];
    const float4 t0 = *(const float4 *)(tile_t<MT>(a.tbuf, tile, NL, 0, 2 * kk) + 4 * lane);
    const float tv0[4] = {t0.x, t0.y, t0.z, t0.w};
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = dY[2 * kk][v] * (1.f - tv0[v] * tv0[v]);
    if (2 * kk + 1 < MT) {
      const int m1 = (2 * kk + 1 < MT) ? 2 * kk + 1 : 0;
      const float4 t1 = *(const float4 *)(tile_t<MT>(a.tbuf, tile, NL, 0, m1) + 4 * lane);
      const float tv1[4] = {t1.x, t1.y, t1.z, t1.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] = dY[m1][v] * (1.f - tv1[v] * tv1[v]);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] = 0.f;
    }
    Bz[kk] = fsplit<P>(x, y);
  }
  // dD one row a of D (16 features b) at a time, contracted with T
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 *Ti = (const float4 *)(a.T32 + (int64_t)(i < 0 ? 0 : i) * M1 * 4);
  float4 Tq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) Tq[r] = i >= 0 ? Ti[4 * g + r] : z4;
  float dT2[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) dT2[r][c] = 0.f;
  // A operands ([aa][kk] blocks of 1 KB) stream through LDS, F0_CA rows of
  // D per chunk, the next chunk loading while this one is used
  const unsigned char *A0 = W + a.fo.a0b[t];
  float4 *dTi = (float4 *)(a.dT32 + (int64_t)(i < 0 ? 0 : i) * M1 * 4);
  const float s = a.inv_nc;
  const int nch = (M1 + F0_CA - 1) / F0_CA;
  dma_blocks(A0, 0, (M1 < F0_CA ? M1 : F0_CA) * KSH, stage[0], wv, lane);
  dma_wait_all();
  for (int aa = 0; aa < M1; ++aa) {
    const int ch = aa / F0_CA, q = aa % F0_CA;
    if (q == 0 && ch + 1 < nch) {
      const int a1 = (ch + 1) * F0_CA, na = (M1 - a1 < F0_CA) ? M1 - a1 : F0_CA;
      dma_blocks(A0, (int64_t)a1 * KSH, na * KSH, stage[(ch + 1) & 1], wv, lane);
    }
    const unsigned char *buf = stage[ch & 1] + q * KSH * 1024;
    v4f c = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < KSH; ++kk) {
      const V av = *(const V *)(buf + kk * 1024 + 16 * lane);
      c = FT<P>::mma(av, Bz[kk].hi, c);
      c = FT<P>::mma(av, Bz[kk].lo, c);
    }
    // c[r] = dE/dD[row n][a = aa][b = 4 g + r]
    const float4 Ta = i >= 0 ? Ti[aa] : z4;
    float4 pc;
    pc.x = c[0] * Tq[0].x + c[1] * Tq[1].x + c[2] * Tq[2].x + c[3] * Tq[3].x;
    pc.y = c[0] * Tq[0].y + c[1] * Tq[1].y + c[2] * Tq[2].y + c[3] * Tq[3].y;
    pc.z = c[0] * Tq[0].z + c[1] * Tq[1].z + c[2] * Tq[2].z + c[3] * Tq[3].z;
    pc.w = c[0] * Tq[0].w + c[1] * Tq[1].w + c[2] * Tq[2].w + c[3] * Tq[3].w;
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
      dT2[r][0] += c[r] * Ta.x;
      dT2[r][1] += c[r] * Ta.y;
      dT2[r][2] += c[r] * Ta.z;
      dT2[r][3] += c[r] * Ta.w;
    }
    if (g == 0) {
      if (aa < 16) sh[wv][n][aa] = pc;
      else if (i >= 0) dTi[aa] = make_float4(pc.x * s, pc.y * s, pc.z * s, pc.w * s);
    }
    if (q == F0_CA - 1 || aa == M1 - 1) dma_wait_all();
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (i >= 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = 4 * g + r;
      if (b < M1) {
        const float4 q = sh[wv][n][b];
        dTi[b] = make_float4((q.x + dT2[r][0]) * s, (q.y + dT2[r][1]) * s, (q.z + dT2[r][2]) * s,
                             (q.w + dT2[r][3]) * s);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
constexpr int FIT_MT = 15;  // hidden width 240

bool fit_mix_supported(const Dims &d, const char **why) {
  const int H = d.fw[1];
  for (int l = 1; l <= d.n_fit; ++l)
    if (d.fw[l] != H) return *why = "mixed fitting net needs equal hidden widths", false;
  if (H != 16 * FIT_MT) return *why = "mixed fitting net is built for hidden width 240", false;
  if (d.M2 != 16) return *why = "mixed fitting net needs M2 = 16", false;
  if (d.M1 % 2 != 0 || d.M1 > 128) return *why = "mixed fitting net needs an even M1 <= 128", false;
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
      fo.ahf[t][l] = put_image(buf, MT, KSH, prec, false, fwd);
      fo.ahb[t][l] = put_image(buf, MT, KSH, prec, false, bwd);
      if (l >= nsplit) {
        fo.ahf_lo[t][l] = put_image(buf, MT, KSH, prec, true, fwd);
        fo.ahb_lo[t][l] = put_image(buf, MT, KSH, prec, true, bwd);
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
  const int64_t tiles = (a.rows + 15) / 16;
  const unsigned grid = (unsigned)((tiles + FIT_WAVES - 1) / FIT_WAVES);
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
