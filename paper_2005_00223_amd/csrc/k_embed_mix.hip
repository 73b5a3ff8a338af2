// Mixed-precision embedding net + descriptor (after the paper's MIX-16
// scheme, Section V-B "Mixed-precision computation"): the embedding layers
// after the first are 16-bit matrix-core products (FP16 or BF16,
// v_mfma_f32_16x16x32) with FP32 accumulation and 16-bit weights; the
// rank-1 first layer, tanh, the skip adds and the descriptor contractions
// stay in FP32; the environment matrix is computed in FP64 and read as FP32
// (the precision every product above takes it in); distances, the force
// Jacobian and every force/virial sum stay in FP64.
//
// Unlike the paper, activations are not rounded to 16 bits: each 16-bit
// operand that carries an activation is split into hi = rn16(x) and
// lo = rn16(x - hi) and multiplied twice (W hi + W lo), which keeps about
// 22 significant bits.  Rounding the activations alone puts the force error
// of the random copper model above 1e-3 eV/A; rounding only the weights
// costs about 4e-5 eV/A (FP16).
//
// Layout.  A wave works on tiles of 16 neighbours; every layer is computed
// transposed (Z^T = W^T H^T, neighbours as the MFMA N dimension).  The f32
// output of v_mfma_f32_16x16x32 leaves lane l with rows 4(l/16)+r (r = 0..3)
// of column l%16, i.e. four consecutive features of one neighbour per
// 16-row tile.  The next layer's B operand needs eight K values of that same
// neighbour per lane, so the K dimension is permuted: k-step kk takes, in
// lane group g = l/16, the features 16(2kk + v/4) + 4g + v%4 (v = 0..7) --
// exactly the registers of output tiles 2kk and 2kk+1.  The host stores the
// weight A operands in this permuted order, lane by lane, so activations go
// from one layer to the next without leaving registers.  Skip partners that
// live in another lane (a doubling skip whose input width is not a multiple
// of 16) are read back from a per-wave LDS copy of the previous layer.
//
// The weights of every (centre type, neighbour type) net are copied into LDS
// once per block.  Per net: w1[32], b1[32] (f32, by slot), A2 [MT2][KS2][64
// lanes][8] (16-bit), b2[S2] (f32), A3 [MT3][KS3][64][8], b3[S3] (f32).
//
// Pass 1: T += G R^T by an LDS transpose of G and v_mfma_f32_16x16x4f32 (K =
// the 16 neighbours), T /= Nc stored in FP32 (the fitting net forms D from
// it).  Pass 2: dE/dT from the fitting net's backward, forward tangent mode
// (h and dh/ds in two MFMA column sets sharing the A operands), then
//   a = G^T dT, b = G'^T dT as split 16-bit MFMAs (hi hi + hi lo + lo hi)
//   with G straight from registers,
//   dE/dR = a + (R . b) e_0, and per 64 neighbours one FP64 pass of
//   g_ij = dE/dR dR/dr, F_i += g, F_j -= g (atomics), Xi -= g (x) r.
#include <cstring>

#include "dp_internal.h"
#include "dp_mix.h"

namespace dpk {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int P> struct HT;
template <> struct HT<0> {
  typedef _Float16 e;
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
};
template <> struct HT<1> {
  typedef __bf16 e;
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
};

template <int P>
__device__ inline v4f mfma16(typename HT<P>::v8 a, typename HT<P>::v8 b, v4f c);
template <>
__device__ inline v4f mfma16<0>(HT<0>::v8 a, HT<0>::v8 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
template <>
__device__ inline v4f mfma16<1>(HT<1>::v8 a, HT<1>::v8 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline v4f mfma32(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <int P>
__device__ inline typename HT<P>::v8 pack8(const float (&x)[4], const float (&y)[4]) {
  typedef typename HT<P>::e E;
  typename HT<P>::v8 v;
  v[0] = (E)x[0]; v[1] = (E)x[1]; v[2] = (E)x[2]; v[3] = (E)x[3];
  v[4] = (E)y[0]; v[5] = (E)y[1]; v[6] = (E)y[2]; v[7] = (E)y[3];
  return v;
}

// hi/lo split of eight activations: x = hi + lo to about 22 bits
template <int P>
struct Split8 {
  typename HT<P>::v8 hi, lo;
};

template <int P>
__device__ inline Split8<P> split8(const float (&x)[4], const float (&y)[4]) {
  typedef typename HT<P>::e E;
  Split8<P> s;
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
__device__ inline Split8<0> split8<0>(const float (&x)[4], const float (&y)[4]) {
  Split8<0> s;
  split8_f16(x, y, s.hi, s.lo);
  return s;
}

__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// skip kind of a layer (in -> out): 0 none, 1 identity, 2 doubling
__host__ __device__ constexpr int skip_kind(int in, int out) { return out == in ? 1 : (out == 2 * in ? 2 : 0); }

template <int W1, int W2, int W3>
struct Shape {
  static constexpr int S1 = 32;                    // layer-1 slots (= K of layer 2)
  static constexpr int S2 = (W2 + 31) / 32 * 32;   // layer-2 slots (= K of layer 3)
  static constexpr int MT2 = S2 / 16;
  static constexpr int KS3 = S2 / 32;
  static constexpr int MT3 = (W3 + 15) / 16;
  static constexpr int S3 = MT3 * 16;
  static constexpr int KSC = (MT3 + 1) / 2;        // k-steps of the contraction over G's slots
  static constexpr int SK1 = (W1 <= 2) ? 1 : 0;    // first layer adds s (out = in or 2 in of a scalar)
  static constexpr int SK2 = skip_kind(W1, W2);
  static constexpr int SK3 = skip_kind(W2, W3);
  // a doubling skip reads another lane's value (through LDS) unless the input
  // width is a multiple of the 16-slot tile
  static constexpr bool XL2 = SK2 == 2 && W1 % 16 != 0;
  static constexpr bool XL3 = SK3 == 2 && W2 % 16 != 0;
  // per-net byte offsets in the LDS copy
  static constexpr int O_W1 = 0, O_B1 = 128, O_A2 = 256;
  static constexpr int O_B2 = O_A2 + MT2 * 1 * 1024;
  static constexpr int O_A3 = O_B2 + S2 * 4;
  static constexpr int O_B3 = O_A3 + MT3 * KS3 * 1024;
  static constexpr int NET_BYTES = O_B3 + S3 * 4;
  // per-wave LDS scratch (bytes)
  static constexpr int P1_H1 = 0;                       // float [16][S1]
  static constexpr int P1_H2 = P1_H1 + 16 * S1 * 4;     // float [16][S2]
  static constexpr int P1_G = P1_H2 + 16 * S2 * 4;      // float [32][GTS]: two output tiles of G, feature-major
  static constexpr int GTS = 20;                        // row stride (neighbours) of that transpose, 16-byte aligned
  static constexpr int P1_R = P1_G + 32 * GTS * 4;      // float [16][4]
  static constexpr int P1_BYTES = P1_R + 256;
  static constexpr int P2_H1 = 0;                       // float [2][16][S1] (h, dh)
  static constexpr int P2_H2 = P2_H1 + 2 * 16 * S1 * 4; // float [2][16][S2]
  static constexpr int P2_R = P2_H2 + 2 * 16 * S2 * 4;  // float [16][4]
  static constexpr int P2_GR = P2_R + 256;              // float [64][4]
  static constexpr int P2_DT = 0;                       // float [S3][4], aliases H1/H2 at the atom's start
  static constexpr int P2_BYTES = P2_GR + 1024;
  static_assert(S3 * 16 <= P2_R, "dT scratch must fit the aliased buffers");
};

constexpr int MIX_WAVES = 4;

// blocks per CU the kernels are compiled for: the student-sized nets leave
// enough registers and LDS for three
template <int W2, int PASS>
struct MixOcc {
  static constexpr int B = (PASS == 1 || W2 <= 32) ? 3 : 2;
};

// rows handled by wave gw of nwaves: a contiguous chunk
__device__ inline void wave_rows(int64_t rows, int64_t &p0, int64_t &p1) {
  const int nw = blockDim.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * nw;
  const int64_t gw = (int64_t)blockIdx.x * nw + (threadIdx.x >> 6);
  const int64_t chunk = (rows + nwaves - 1) / nwaves;
  p0 = gw * chunk;
  p1 = p0 + chunk < rows ? p0 + chunk : rows;
}

__device__ inline void copy_nets(unsigned char *dst, const unsigned char *src, int bytes) {
  const uint4 *s = (const uint4 *)src;
  uint4 *d = (uint4 *)dst;
  for (int o = threadIdx.x; o < bytes / 16; o += blockDim.x) d[o] = s[o];
}

// Environment row of slot q of a type block of cnt >= 1 real slots: the
// load is unconditional (a slot past the block reads the last real row and
// returns zeros), so it never waits behind a branch.
__device__ inline float4 rt_row(const float4 *rt, int64_t base, int q, int cnt) {
  const float4 v = rt[base + (q < cnt ? q : cnt - 1)];
  return q < cnt ? v : make_float4(0.f, 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// T += G R^T over the 16 neighbours of a tile, G transposed through LDS.
// FP16: v_mfma_f32_16x16x16_f16 with G and R as hi + lo halves (three
// products, about 22 bits); BF16 (8-bit halves would lose bits): the FP32
// matrix core, v_mfma_f32_16x16x4f32 over four K-steps of 4 neighbours.
// ---------------------------------------------------------------------------
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
struct RSplit {
  f16x4 hi, lo;
};

__device__ inline void split4_f16(float4 v, f16x4 &hi, f16x4 &lo) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  const h2 p0 = {(_Float16)v.x, (_Float16)v.y}, p1 = {(_Float16)v.z, (_Float16)v.w};
  const unsigned H0 = __builtin_bit_cast(unsigned, p0), H1 = __builtin_bit_cast(unsigned, p1);
  const u2 hv = {H0, H1}, lv = {f16_lo_pair(v.x, v.y, H0), f16_lo_pair(v.z, v.w, H1)};
  hi = __builtin_bit_cast(f16x4, hv);
  lo = __builtin_bit_cast(f16x4, lv);
}

// lane (g, n): R[4g + v][c = n] for n < 4, else 0
template <int P>
__device__ inline RSplit rsplit(const float *Rs, int n, int g) {
  RSplit r;
  if (P == 0) {
    float4 v;
    v.x = n < 4 ? Rs[4 * (4 * g + 0) + n] : 0.f;
    v.y = n < 4 ? Rs[4 * (4 * g + 1) + n] : 0.f;
    v.z = n < 4 ? Rs[4 * (4 * g + 2) + n] : 0.f;
    v.w = n < 4 ? Rs[4 * (4 * g + 3) + n] : 0.f;
    split4_f16(v, r.hi, r.lo);
  }
  return r;
}

// grow = G^T row of feature 16 mt + n in the LDS transpose (neighbours
// contiguous); returns acc + G^T R for output tile mt, lane layout of T
template <int P>
__device__ inline v4f tacc16(const float *grow, const RSplit &RB, const float *Rs, int n, int g, v4f acc) {
  if (P == 0) {
    f16x4 ahi, alo;
    split4_f16(*(const float4 *)(grow + 4 * g), ahi, alo);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, RB.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, RB.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(alo, RB.hi, acc, 0, 0, 0);
  } else {
    // K-step kk: neighbours 4kk..4kk+3, lane (g, n) supplies G[4kk + g][16mt + n] and R[4kk + g][n]
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const float rb = n < 4 ? Rs[4 * (4 * kk + g) + n] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(grow[4 * kk + g], rb, acc, 0, 0, 0);
    }
  }
  return acc;
}

// The same row scaled by 0 past the block instead of selected: the load's
// result is always used, so the compiler keeps it unconditional and in
// flight.
__device__ inline float4 rt_row_m(const float4 *rt, int64_t base, int q, int cnt) {
  const float4 v = rt[base + (q < cnt ? q : cnt - 1)];
  const float m = q < cnt ? 1.f : 0.f;
  return make_float4(v.x * m, v.y * m, v.z * m, v.w * m);
}

// x, y, z of atom j; w (the type) is not loaded: a dead part of a load in
// flight lets the compiler reuse its registers only after waiting for it
__device__ inline double4 pos3(const double4 *xw, int j) {
  const double2 xy = *(const double2 *)(xw + j);
  const double z = ((const double *)(xw + j))[2];
  return make_double4(xy.x, xy.y, z, 0.0);
}

// ---------------------------------------------------------------------------
// layer 1 on VALU: lane (g, n) computes slots 16 mt + 4 g + r (mt < 2)
// ---------------------------------------------------------------------------
template <int W1, bool TANGENT>
__device__ inline void layer1(const float *w1, const float *b1, float s, int g, float (&h)[2][4], float (&hd)[2][4]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const float4 w = *(const float4 *)(w1 + 16 * mt + 4 * g);
    const float4 b = *(const float4 *)(b1 + 16 * mt + 4 * g);
    const float wv[4] = {w.x, w.y, w.z, w.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (16 * mt >= W1) {  // whole tile is padding (compile-time)
        h[mt][r] = 0.f;
        hd[mt][r] = 0.f;
        continue;
      }
      const int f = 16 * mt + 4 * g + r;
      const float t = tanh_f(s * wv[r] + bv[r]);
      float hv = t, dv = (1.f - t * t) * wv[r];
      if (W1 <= 2) {
        hv += s;
        dv += 1.f;
      }
      h[mt][r] = f < W1 ? hv : 0.f;
      if (TANGENT) hd[mt][r] = f < W1 ? dv : 0.f;
    }
  }
}

// one MFMA layer from 16-bit weights in LDS; acc initialised with the bias;
// B holds the hi/lo split activations of each k-step
template <int P, int MT, int KS>
__device__ inline void layer_mfma(const unsigned char *Aops, const float *bias, const Split8<P> (&B)[KS], int lane,
                                  int g, v4f (&acc)[MT]) {
  typedef typename HT<P>::v8 V;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const float4 b = *(const float4 *)(bias + 16 * mt + 4 * g);
    acc[mt] = v4f{b.x, b.y, b.z, b.w};
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const V a = *(const V *)(Aops + ((mt * KS + kk) * 64 + lane) * 16);
      acc[mt] = mfma16<P>(a, B[kk].hi, acc[mt]);
      acc[mt] = mfma16<P>(a, B[kk].lo, acc[mt]);
    }
}

// one output tile mt of an MFMA layer (bias-initialised when bias != NULL)
template <int P, int KS>
__device__ inline v4f mfma_tile(const unsigned char *Aops, const float *bias, const Split8<P> (&B)[KS], int lane,
                                int g, int mt) {
  typedef typename HT<P>::v8 V;
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  if (bias) {
    const float4 b = *(const float4 *)(bias + 16 * mt + 4 * g);
    acc = v4f{b.x, b.y, b.z, b.w};
  }
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const V a = *(const V *)(Aops + ((mt * KS + kk) * 64 + lane) * 16);
    acc = mfma16<P>(a, B[kk].hi, acc);
    acc = mfma16<P>(a, B[kk].lo, acc);
  }
  return acc;
}

// tangent columns: same A operands, zero initial accumulator
template <int P, int MT, int KS>
__device__ inline void layer_mfma_tan(const unsigned char *Aops, const Split8<P> (&B)[KS], int lane, v4f (&acc)[MT]) {
  typedef typename HT<P>::v8 V;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const V a = *(const V *)(Aops + ((mt * KS + kk) * 64 + lane) * 16);
      acc[mt] = mfma16<P>(a, B[kk].hi, acc[mt]);
      acc[mt] = mfma16<P>(a, B[kk].lo, acc[mt]);
    }
}

// value of the previous layer added by the skip connection for output
// feature f of lane (g, n): the same register when f < IN, the LDS copy
// otherwise (doubling skip); 0 when the layer has no skip.
template <int IN, int OUT, int SK, int MTI>
__device__ inline float skip_val(int f, int mt, int r, const float (&prev)[MTI][4], const float *prev_lds, int n,
                                 int stride) {
  if (SK == 0 || f >= OUT) return 0.f;
  if (SK == 1) return (mt < MTI) ? prev[mt < MTI ? mt : 0][r] : 0.f;
  // doubling
  float own = (mt < MTI) ? prev[mt < MTI ? mt : 0][r] : 0.f;
  if constexpr (IN % 16 == 0) {
    // partner slot f - IN = 16 (mt - IN/16) + 4 g + r is held by this lane
    constexpr int DM = IN / 16;
    const int ms = mt - DM;
    const float part = (ms >= 0 && ms < MTI) ? prev[(ms >= 0 && ms < MTI) ? ms : 0][r] : 0.f;
    return f < IN ? own : part;
  }
  const int src = f >= IN ? f - IN : 0;
  const float other = prev_lds[n * stride + src];
  return f < IN ? own : other;
}

// LIN: the last layer is affine (no tanh), as in the student nets
template <int W1, int W2, int W3, int LIN, int P>
__global__ void __launch_bounds__(64 * MIX_WAVES, (MixOcc<W2, 1>::B)) k_embed_fwd_mix(MixArgs a) {
  typedef Shape<W1, W2, W3> S;
  extern __shared__ __align__(16) unsigned char smem[];
  const Dims &d = a.d;
  const int nnets = d.ntypes * d.ntypes;
  copy_nets(smem, a.nets, nnets * S::NET_BYTES);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  unsigned char *ws = smem + nnets * S::NET_BYTES + wv * S::P1_BYTES;
  float *h1s = (float *)(ws + S::P1_H1);
  float *h2s = (float *)(ws + S::P1_H2);
  float *Gs = (float *)(ws + S::P1_G);
  float *Rs = (float *)(ws + S::P1_R);
  int64_t p0, p1;
  wave_rows(a.rows, p0, p1);
  for (int64_t p = p0; p < p1; ++p) {
    const int i = a.atom_of_pos[p];
    if (i < 0) continue;
    const int t = (int)a.xw[i].w;
    v4f Tacc[S::MT3];
#pragma unroll
    for (int mt = 0; mt < S::MT3; ++mt) Tacc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int u = 0; u < d.ntypes; ++u) {
      const unsigned char *net = smem + (t * d.ntypes + u) * S::NET_BYTES;
      const float *w1 = (const float *)(net + S::O_W1), *b1 = (const float *)(net + S::O_B1);
      const float *b2 = (const float *)(net + S::O_B2), *b3 = (const float *)(net + S::O_B3);
      const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
      const int64_t base = (int64_t)i * d.nnei + d.off[u];
      for (int n0 = 0; n0 < cnt; n0 += 16) {
        const float4 r4 = rt_row(a.rt, base, n0 + n, cnt);
        const float s = r4.x;
        if (g == 0) *(float4 *)(Rs + 4 * n) = make_float4(r4.x, r4.y, r4.z, r4.w);
        float h1[2][4], hd_unused[2][4];
        layer1<W1, false>(w1, b1, s, g, h1, hd_unused);
        if (S::XL2)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
            *(float4 *)(h1s + n * S::S1 + 16 * mt + 4 * g) = make_float4(h1[mt][0], h1[mt][1], h1[mt][2], h1[mt][3]);
        Split8<P> B2[1] = {split8<P>(h1[0], h1[1])};
        v4f acc2[S::MT2];
        layer_mfma<P, S::MT2, 1>(net + S::O_A2, b2, B2, lane, g, acc2);
        wsync();
        // R of the tile's neighbours 4g..4g+3, component n, as the B operand of T += G R^T
        const RSplit RB = rsplit<P>(Rs, n, g);
        float h2[S::MT2][4];
#pragma unroll
        for (int mt = 0; mt < S::MT2; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int f = 16 * mt + 4 * g + r;
            float v = 0.f;
            if (16 * mt < W2 && f < W2) v = tanh_f(acc2[mt][r]) + skip_val<W1, W2, S::SK2, 2>(f, mt, r, h1, h1s, n, S::S1);
            h2[mt][r] = v;
          }
        if (S::XL3)
#pragma unroll
          for (int mt = 0; mt < S::MT2; ++mt)
            *(float4 *)(h2s + n * S::S2 + 16 * mt + 4 * g) = make_float4(h2[mt][0], h2[mt][1], h2[mt][2], h2[mt][3]);
        Split8<P> B3[S::KS3];
#pragma unroll
        for (int kk = 0; kk < S::KS3; ++kk) B3[kk] = split8<P>(h2[2 * kk], h2[2 * kk + 1]);
        wsync();
        // layer 3, G and T += G R^T, one pair of output tiles at a time
#pragma unroll
        for (int kp = 0; kp < S::KSC; ++kp) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int mt = 2 * kp + q;
            float gv[4] = {0.f, 0.f, 0.f, 0.f};
            if (mt < S::MT3) {
              const v4f acc3 = mfma_tile<P, S::KS3>(net + S::O_A3, b3, B3, lane, g, mt);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int f = 16 * mt + 4 * g + r;
                if (f < W3)
                  gv[r] = (LIN ? acc3[r] : tanh_f(acc3[r])) + skip_val<W2, W3, S::SK3, S::MT2>(f, mt, r, h2, h2s, n, S::S2);
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Gs[(16 * q + 4 * g + r) * S::GTS + n] = gv[r];
          }
          wsync();
          // T[f][c] += sum_nb G[nb][f] R[nb][c] over the tile's 16 neighbours:
          // A = G^T (rows f, K = neighbours), B = R (K = neighbours, N = c)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            if (2 * kp + q < S::MT3) {
              Tacc[2 * kp + q] = tacc16<P>(Gs + (16 * q + n) * S::GTS, RB, Rs, n, g, Tacc[2 * kp + q]);
            }
          }
          wsync();
        }
      }
    }
    // T / Nc: lane (g, n) holds T[16 mt + 4 g + r][n] for n < 4; the
    // fitting net forms D = T T_<^T itself
    float *Tg = a.T32 + (int64_t)i * d.M1 * 4;
#pragma unroll
    for (int mt = 0; mt < S::MT3; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = 16 * mt + 4 * g + r;
        if (n < 4 && f < d.M1) Tg[4 * f + n] = Tacc[mt][r] * (float)d.inv_nc;
      }
  }
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
// pair_force with the neighbour's share scattered by global atomics;
// D4 = (d, r^2) of the pair and j = nlist[slot]
__device__ inline void force_pair(const MixArgs &a, int64_t slot, const double4 &D4, int j, float4 gr, double rc,
                                  double rcs, double inv_w, double &fi0, double &fi1, double &fi2, double (&vir)[9]) {
  if (a.net_deriv) {
    double *nd = a.net_deriv + slot * 4;
    nd[0] = gr.x; nd[1] = gr.y; nd[2] = gr.z; nd[3] = gr.w;
  }
  double gx, gy, gz;
  pair_force(D4, gr, rc, rcs, inv_w, gx, gy, gz, fi0, fi1, fi2, vir);
  unsafeAtomicAdd(a.force + 3 * (int64_t)j + 0, -gx);
  unsafeAtomicAdd(a.force + 3 * (int64_t)j + 1, -gy);
  unsafeAtomicAdd(a.force + 3 * (int64_t)j + 2, -gz);
}

// wave sum of the centre atom's force, one atomic per component
__device__ inline void finish_atom_force(const MixArgs &a, int i, int lane, double fi0, double fi1, double fi2) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    fi0 += __shfl_xor(fi0, o);
    fi1 += __shfl_xor(fi1, o);
    fi2 += __shfl_xor(fi2, o);
  }
  if (lane == 0) {
    unsafeAtomicAdd(a.force + 3 * (int64_t)i + 0, fi0);
    unsafeAtomicAdd(a.force + 3 * (int64_t)i + 1, fi1);
    unsafeAtomicAdd(a.force + 3 * (int64_t)i + 2, fi2);
  }
}

// block partial of the virial (fixed order: lanes, then waves)
__device__ inline void finish_block_virial(const MixArgs &a, const double (&vir)[9], double (&vred)[MIX_WAVES][9],
                                           int lane, int wv) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double v = vir[k];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    if (lane == 0) vred[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double v = 0.0;
    for (int w = 0; w < MIX_WAVES; ++w) v += vred[w][threadIdx.x];
    a.vir_part[(int64_t)blockIdx.x * 9 + threadIdx.x] = v;
  }
}

template <int W1, int W2, int W3, int LIN, int P>
__global__ void __launch_bounds__(64 * MIX_WAVES, (MixOcc<W2, 2>::B)) k_embed_bwd_mix(MixArgs a) {
  typedef Shape<W1, W2, W3> S;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double vred[MIX_WAVES][9];
  const Dims &d = a.d;
  const int nnets = d.ntypes * d.ntypes;
  copy_nets(smem, a.nets, nnets * S::NET_BYTES);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  unsigned char *ws = smem + nnets * S::NET_BYTES + wv * S::P2_BYTES;
  float *h1s = (float *)(ws + S::P2_H1), *hd1s = h1s + 16 * S::S1;
  float *h2s = (float *)(ws + S::P2_H2), *hd2s = h2s + 16 * S::S2;
  float *Rs = (float *)(ws + S::P2_R);
  float *gRs = (float *)(ws + S::P2_GR);
  float *dTs = (float *)(ws + S::P2_DT);
  const double rc = d.rcut, rcs = d.rcut_smth, inv_w = 1.0 / (d.rcut - d.rcut_smth);
  double vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0;
  int64_t p0, p1;
  wave_rows(a.rows, p0, p1);
  for (int64_t p = p0; p < p1; ++p) {
    const int i = a.atom_of_pos[p];
    if (i < 0) continue;
    const double4 xi = a.xw[i];
    const int t = (int)xi.w;
    // dE/dT of the unscaled sum (from the fitting net) in LDS, rows f >= M1 zero
    {
      const float *dTi = a.dT32 + (int64_t)i * d.M1 * 4;
      for (int o = lane; o < S::S3 * 4; o += 64) dTs[o] = (o >> 2) < d.M1 ? dTi[o] : 0.f;
    }
    wsync();
    // B operand of the contraction: K = G's slots (permuted as the layer chain), N = components
    Split8<P> dTB[S::KSC];
#pragma unroll
    for (int kk = 0; kk < S::KSC; ++kk) {
      float x[4], y[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int f0 = 16 * (2 * kk) + 4 * g + v, f1 = 16 * (2 * kk + 1) + 4 * g + v;
        x[v] = (n < 4 && f0 < S::S3) ? dTs[4 * f0 + n] : 0.f;
        y[v] = (n < 4 && f1 < S::S3) ? dTs[4 * f1 + n] : 0.f;
      }
      dTB[kk] = split8<P>(x, y);
    }
    wsync();
    double fi0 = 0.0, fi1 = 0.0, fi2 = 0.0;
    for (int u = 0; u < d.ntypes; ++u) {
      const unsigned char *net = smem + (t * d.ntypes + u) * S::NET_BYTES;
      const float *w1 = (const float *)(net + S::O_W1), *b1 = (const float *)(net + S::O_B1);
      const float *b2 = (const float *)(net + S::O_B2), *b3 = (const float *)(net + S::O_B3);
      const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
      const int64_t base = (int64_t)i * d.nnei + d.off[u];
      for (int n0 = 0; n0 < cnt; n0 += 16) {
        const float4 r4 = rt_row(a.rt, base, n0 + n, cnt);
        const float s = r4.x;
        if (g == 0) *(float4 *)(Rs + 4 * n) = make_float4(r4.x, r4.y, r4.z, r4.w);
        float h1[2][4], hd1[2][4];
        layer1<W1, true>(w1, b1, s, g, h1, hd1);
        if (S::XL2)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            *(float4 *)(h1s + n * S::S1 + 16 * mt + 4 * g) = make_float4(h1[mt][0], h1[mt][1], h1[mt][2], h1[mt][3]);
            *(float4 *)(hd1s + n * S::S1 + 16 * mt + 4 * g) =
                make_float4(hd1[mt][0], hd1[mt][1], hd1[mt][2], hd1[mt][3]);
          }
        Split8<P> B2h[1] = {split8<P>(h1[0], h1[1])}, B2d[1] = {split8<P>(hd1[0], hd1[1])};
        v4f acc2[S::MT2], acc2d[S::MT2];
        layer_mfma<P, S::MT2, 1>(net + S::O_A2, b2, B2h, lane, g, acc2);
        layer_mfma_tan<P, S::MT2, 1>(net + S::O_A2, B2d, lane, acc2d);
        wsync();
        float h2[S::MT2][4], hd2[S::MT2][4];
#pragma unroll
        for (int mt = 0; mt < S::MT2; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int f = 16 * mt + 4 * g + r;
            float hv = 0.f, dv = 0.f;
            if (16 * mt < W2 && f < W2) {
              const float th = tanh_f(acc2[mt][r]);
              hv = th + skip_val<W1, W2, S::SK2, 2>(f, mt, r, h1, h1s, n, S::S1);
              dv = (1.f - th * th) * acc2d[mt][r] + skip_val<W1, W2, S::SK2, 2>(f, mt, r, hd1, hd1s, n, S::S1);
            }
            h2[mt][r] = hv;
            hd2[mt][r] = dv;
          }
        if (S::XL3)
#pragma unroll
          for (int mt = 0; mt < S::MT2; ++mt) {
            *(float4 *)(h2s + n * S::S2 + 16 * mt + 4 * g) = make_float4(h2[mt][0], h2[mt][1], h2[mt][2], h2[mt][3]);
            *(float4 *)(hd2s + n * S::S2 + 16 * mt + 4 * g) =
                make_float4(hd2[mt][0], hd2[mt][1], hd2[mt][2], hd2[mt][3]);
          }
        Split8<P> B3h[S::KS3], B3d[S::KS3];
#pragma unroll
        for (int kk = 0; kk < S::KS3; ++kk) {
          B3h[kk] = split8<P>(h2[2 * kk], h2[2 * kk + 1]);
          B3d[kk] = split8<P>(hd2[2 * kk], hd2[2 * kk + 1]);
        }
        wsync();
        // layer 3 with tangent, then a = G^T dT and b = G'^T dT, one pair of
        // output tiles at a time (G and G' never leave registers)
        v4f ca = v4f{0.f, 0.f, 0.f, 0.f}, cb = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kp = 0; kp < S::KSC; ++kp) {
          float G[2][4], Gd[2][4];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int mt = 2 * kp + q;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              G[q][r] = 0.f;
              Gd[q][r] = 0.f;
            }
            if (mt < S::MT3) {
              const v4f h3 = mfma_tile<P, S::KS3>(net + S::O_A3, b3, B3h, lane, g, mt);
              const v4f d3 = mfma_tile<P, S::KS3>(net + S::O_A3, nullptr, B3d, lane, g, mt);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int f = 16 * mt + 4 * g + r;
                if (f < W3) {
                  const float th = LIN ? h3[r] : tanh_f(h3[r]);
                  G[q][r] = th + skip_val<W2, W3, S::SK3, S::MT2>(f, mt, r, h2, h2s, n, S::S2);
                  Gd[q][r] = (LIN ? d3[r] : (1.f - th * th) * d3[r]) +
                             skip_val<W2, W3, S::SK3, S::MT2>(f, mt, r, hd2, hd2s, n, S::S2);
                }
              }
            }
          }
          const Split8<P> ga = split8<P>(G[0], G[1]);
          const Split8<P> gb = split8<P>(Gd[0], Gd[1]);
          ca = mfma16<P>(ga.hi, dTB[kp].hi, ca);
          ca = mfma16<P>(ga.hi, dTB[kp].lo, ca);
          ca = mfma16<P>(ga.lo, dTB[kp].hi, ca);
          cb = mfma16<P>(gb.hi, dTB[kp].hi, cb);
          cb = mfma16<P>(gb.hi, dTB[kp].lo, cb);
          cb = mfma16<P>(gb.lo, dTB[kp].hi, cb);
        }
        const int slot0 = n0 & 63;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int nb = 4 * g + r;
          float pr = n < 4 ? Rs[4 * nb + n] * cb[r] : 0.f;
          pr += __shfl_xor(pr, 1);
          pr += __shfl_xor(pr, 2);
          const float gr = ca[r] + (n == 0 ? pr : 0.f);
          if (n < 4) gRs[4 * (slot0 + nb) + n] = gr;
        }
        wsync();
        // every 64 neighbours (or at the end of the type block): FP64 force pass
        if (((n0 + 16) & 63) == 0 || n0 + 16 >= cnt) {
          const int c0 = n0 & ~63;
          const int q = c0 + lane;
          if (q < cnt) {
            const float4 gr = *(const float4 *)(gRs + 4 * lane);
            const int j = a.nlist[base + q];
            force_pair(a, base + q, pair_disp_sq(xi, a.xw[j], a.L[0], a.L[1], a.L[2]), j, gr, rc, rcs, inv_w, fi0,
                       fi1, fi2, vir);
          }
          wsync();
        }
      }
    }
    finish_atom_force(a, i, lane, fi0, fi1, fi2);
  }
  finish_block_virial(a, vir, vred, lane, wv);
}

// ---------------------------------------------------------------------------
// affine last layer (the student nets): G = W3^T h2 + b3 is linear in h2, so
//   T   = sum_nb G R^T = W3^T (sum_nb h2 R^T) + b3 (sum_nb R)^T
//   G^T dT  = h2^T (W3 dT) + b3^T dT,   G'^T dT = h2'^T (W3 dT)
// and the third layer leaves the per-neighbour work: per neighbour only the
// 32 x 4 sum H = sum h2 R^T (pass 1) or the contraction with the 32 x 4
// matrix M = W3 dT (pass 2) remains, W3 is applied once per (atom, net).
// H in its MFMA accumulator layout is exactly the K-permuted B operand of the
// layer-3 image W3^T, and M in its accumulator layout is exactly the A
// operand of the per-neighbour contraction.
// ---------------------------------------------------------------------------
// Tabulated second layer at s (0 <= s <= the table's range): lane group g
// gets features f = 16 mt + 4 g + r, r = 0..3 (the MFMA output layout);
// cubic Hermite interpolation between rows k and k + 1, written with the
// node difference y1 - y0 (h00 = 1 - h01) so that value and slope share it;
// D: also ds * dh2/ds (the caller applies the factor 1/ds once per neighbour).
template <bool D>
__device__ inline void tab_h2(const float *tab, float s, float inv_ds, int g, float (&h)[2][4], float (&dh)[2][4]) {
  const float x = s * inv_ds;
  int k = (int)x;
  k = k < TAB_K - 1 ? k : TAB_K - 1;
  const float t = x - (float)k, t2 = t * t, t3 = t2 * t;
  const float h10 = t3 - 2.f * t2 + t, h01 = 3.f * t2 - 2.f * t3, h11 = t3 - t2;
  const float e01 = 6.f * (t - t2), e10 = 3.f * t2 - 4.f * t + 1.f, e11 = 3.f * t2 - 2.f * t;
  const float *r0 = tab + k * TAB_STRIDE, *r1 = r0 + TAB_STRIDE;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int c = 2 * (16 * mt + 4 * g);
    const float4 a0 = *(const float4 *)(r0 + c), a1 = *(const float4 *)(r0 + c + 4);
    const float4 b0 = *(const float4 *)(r1 + c), b1 = *(const float4 *)(r1 + c + 4);
    const float y0[4] = {a0.x, a0.z, a1.x, a1.z}, m0[4] = {a0.y, a0.w, a1.y, a1.w};
    const float y1[4] = {b0.x, b0.z, b1.x, b1.z}, m1[4] = {b0.y, b0.w, b1.y, b1.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float dy = y1[r] - y0[r];
      h[mt][r] = h01 * dy + h10 * m0[r] + h11 * m1[r] + y0[r];
      if (D) dh[mt][r] = e01 * dy + e10 * m0[r] + e11 * m1[r];
    }
  }
}

template <int W1, int W2, int W3>
struct LinShape {
  typedef Shape<W1, W2, W3> S;
  static_assert(S::S2 == 32 && S::KS3 == 1, "affine kernels take the 32-slot second layer as one K-step");
  static_assert(S::SK3 == 0, "affine kernels assume no skip into the last layer");
  static constexpr int KF = (W3 + 31) / 32;             // K-steps of M = W3 dT over the outputs
  static constexpr int O_A3B = S::NET_BYTES;            // W3 as [k][f] A operands: [2][KF][64 lanes][8]
  static constexpr int NET_BYTES = O_A3B + 2 * KF * 1024;
  static constexpr int XL = S::XL2 ? 1 : 0;             // cross-lane skip scratch needed
  static constexpr int P1_H1 = 0;                       // float [16][S1] (cross-lane skips only)
  static constexpr int P1_HT = P1_H1 + XL * 16 * S::S1 * 4;  // float [32][GTS]: h2 transposed (features x neighbours)
  static constexpr int P1_R = P1_HT + 32 * S::GTS * 4;  // float [16][4]
  static constexpr int P1_BYTES = P1_R + 256;
  static constexpr int P2_H1 = 0;                       // float [2][16][S1] (h, dh; cross-lane skips only)
  static constexpr int DT_ROWS = KF * 32;              // rows of dT read by the K-steps of W3 dT (zero past M1)
  static constexpr int P2_DT = P2_H1 + XL * 2 * 16 * S::S1 * 4;  // float [DT_ROWS][4]
  static constexpr int P2_GR = P2_DT + DT_ROWS * 16;    // float [64][4]
  // per wave: the above (layers), or the projected table (dT staged in it first)
  static constexpr int P2_BYTES = P2_GR + 1024 > PT_BYTES ? P2_GR + 1024 : PT_BYTES;
  static_assert(DT_ROWS * 16 <= PT_BYTES, "dT is staged in the projected table's scratch");
};

template <int W1, int W2, int W3, int P>
__global__ void __launch_bounds__(64 * MIX_WAVES, 3) k_embed_fwd_lin(MixArgs a) {
  typedef Shape<W1, W2, W3> S;
  typedef LinShape<W1, W2, W3> LS;
  extern __shared__ __align__(16) unsigned char smem[];
  const Dims &d = a.d;
  const int nnets = d.ntypes * d.ntypes;
  copy_nets(smem, a.nets, nnets * LS::NET_BYTES);
  const int tab_bytes = a.tab ? nnets * TAB_BYTES : 0;  // student table after the nets
  if (a.tab) copy_nets(smem + nnets * LS::NET_BYTES, (const unsigned char *)a.tab, tab_bytes);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  const float *tabs = (const float *)(smem + nnets * LS::NET_BYTES);
  unsigned char *ws = smem + nnets * LS::NET_BYTES + tab_bytes + wv * LS::P1_BYTES;
  float *h1s = (float *)(ws + LS::P1_H1);
  float *Hs = (float *)(ws + LS::P1_HT);
  float *Rs = (float *)(ws + LS::P1_R);
  int64_t p0, p1;
  wave_rows(a.rows, p0, p1);
  for (int64_t p = p0; p < p1; ++p) {
    const int i = a.atom_of_pos[p];
    if (i < 0) continue;
    const int t = (int)a.xw[i].w;
    v4f Tacc[S::MT3];
#pragma unroll
    for (int mt = 0; mt < S::MT3; ++mt) Tacc[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int u = 0; u < d.ntypes; ++u) {
      const unsigned char *net = smem + (t * d.ntypes + u) * LS::NET_BYTES;
      const float *w1 = (const float *)(net + S::O_W1), *b1 = (const float *)(net + S::O_B1);
      const float *b2 = (const float *)(net + S::O_B2), *b3 = (const float *)(net + S::O_B3);
      const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
      if (cnt == 0) continue;
      const int64_t base = (int64_t)i * d.nnei + d.off[u];
      v4f Hacc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
      float sr0 = 0.f, sr1 = 0.f, sr2 = 0.f, sr3 = 0.f;  // this lane's neighbours: sum of R
      float4 r4n = rt_row(a.rt, base, n, cnt);
      for (int n0 = 0; n0 < cnt; n0 += 16) {
        // this tile's environment rows; the next tile's are loaded meanwhile
        const float4 r4 = r4n;
        if (n0 + 16 < cnt) r4n = rt_row(a.rt, base, n0 + 16 + n, cnt);
        const float s = r4.x;
        if (g == 0) *(float4 *)(Rs + 4 * n) = make_float4(r4.x, r4.y, r4.z, r4.w);
        sr0 += r4.x;
        sr1 += r4.y;
        sr2 += r4.z;
        sr3 += r4.w;
        float h2[2][4];
        if (a.tab && __ballot(s > a.tab_shi) == 0ull) {
          // every neighbour of the tile inside the table's range
          float unused[2][4];
          tab_h2<false>(tabs + (t * d.ntypes + u) * (TAB_BYTES / 4), s, a.tab_inv_ds, g, h2, unused);
        } else {
          float h1[2][4], hd_unused[2][4];
          layer1<W1, false>(w1, b1, s, g, h1, hd_unused);
          if (S::XL2)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
              *(float4 *)(h1s + n * S::S1 + 16 * mt + 4 * g) =
                  make_float4(h1[mt][0], h1[mt][1], h1[mt][2], h1[mt][3]);
          Split8<P> B2[1] = {split8<P>(h1[0], h1[1])};
          v4f acc2[S::MT2];
          layer_mfma<P, S::MT2, 1>(net + S::O_A2, b2, B2, lane, g, acc2);
          wsync();
#pragma unroll
          for (int mt = 0; mt < S::MT2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int f = 16 * mt + 4 * g + r;
              float v = 0.f;
              if (16 * mt < W2 && f < W2)
                v = tanh_f(acc2[mt][r]) + skip_val<W1, W2, S::SK2, 2>(f, mt, r, h1, h1s, n, S::S1);
              h2[mt][r] = v;
            }
        }
        // h2, written transposed (features x neighbours) for H += h2^T R
#pragma unroll
        for (int mt = 0; mt < S::MT2; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) Hs[(16 * mt + 4 * g + r) * S::GTS + n] = h2[mt][r];
        wsync();
        const RSplit RB = rsplit<P>(Rs, n, g);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) Hacc[mt] = tacc16<P>(Hs + (16 * mt + n) * S::GTS, RB, Rs, n, g, Hacc[mt]);
        wsync();
      }
      // T += W3^T H: H (lane (g, n): H[16 mt + 4 g + r][c = n]) is the K-permuted B operand
      float hx[4], hy[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        hx[r] = Hacc[0][r];
        hy[r] = Hacc[1][r];
      }
      const Split8<P> HB[1] = {split8<P>(hx, hy)};
#pragma unroll
      for (int mt = 0; mt < S::MT3; ++mt) {
        const v4f z = mfma_tile<P, 1>(net + S::O_A3, nullptr, HB, lane, g, mt);
        Tacc[mt] += z;
      }
      // + b3 (sum R)^T: sum over the 16 neighbour lanes of a row, component c = n
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        sr0 += __shfl_xor(sr0, o);
        sr1 += __shfl_xor(sr1, o);
        sr2 += __shfl_xor(sr2, o);
        sr3 += __shfl_xor(sr3, o);
      }
      const float src = n == 0 ? sr0 : (n == 1 ? sr1 : (n == 2 ? sr2 : (n == 3 ? sr3 : 0.f)));
#pragma unroll
      for (int mt = 0; mt < S::MT3; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int f = 16 * mt + 4 * g + r;
          if (f < W3) Tacc[mt][r] += b3[f] * src;
        }
    }
    float *Tg = a.T32 + (int64_t)i * d.M1 * 4;
#pragma unroll
    for (int mt = 0; mt < S::MT3; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = 16 * mt + 4 * g + r;
        if (n < 4 && f < d.M1) Tg[4 * f + n] = Tacc[mt][r] * (float)d.inv_nc;
      }
  }
}

// FP64 add into the block's LDS accumulator, through an LDS-qualified
// pointer: the compiler then never merges it with the global atomics of the
// other branch into one atomic on a pointer of unknown kind
typedef __attribute__((address_space(3))) double lds_f64;
__device__ inline void lds_add(double *p, double v) {
  __hip_atomic_fetch_add((lds_f64 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS force accumulation of the cell-ordered backward: the block owns one
// cell of the list grid, facc[27][cap][3] holds the forces on the atoms of the
// 27 cells around it (slot = offset (dx, dy, dz) in {-1, 0, 1}^3, then the
// atom's index inside its cell)
struct CellCtx {
  double *facc;
  const uint32_t *code;   // per atom: cx << 24 | cy << 16 | cz << 8 | min(index in cell, 255)
  int cx, cy, cz, nc0, nc1, nc2, cap;
};

// LDS slot of an atom with cell code `code`, or -1 when it lies outside the
// 27 cells or past the capacity (its force then goes to global memory)
__device__ inline int cell_slot(const CellCtx &cc, uint32_t code) {
  int dx = (int)(code >> 24) - cc.cx, dy = (int)((code >> 16) & 255u) - cc.cy, dz = (int)((code >> 8) & 255u) - cc.cz;
  if (dx > 1) dx -= cc.nc0;
  else if (dx < -1) dx += cc.nc0;
  if (dy > 1) dy -= cc.nc1;
  else if (dy < -1) dy += cc.nc1;
  if (dz > 1) dz -= cc.nc2;
  else if (dz < -1) dz += cc.nc2;
  const int l = (int)(code & 255u);
  if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1 || l >= cc.cap) return -1;
  return ((dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)) * cc.cap + l;
}

// h2 and ds-derivative of the second layer by the layers themselves, for the
// 16 neighbours of a tile (lane (g, n): features 16 mt + 4 g + r of
// neighbour n at s); h1s / hd1s: the cross-lane skip scratch (XL2 shapes)
template <int W1, int W2, int W3, int P>
__device__ inline void layers_h2(const unsigned char *net, float s, int lane, float *h1s, float *hd1s,
                                 float (&h2)[Shape<W1, W2, W3>::MT2][4], float (&hd2)[Shape<W1, W2, W3>::MT2][4]) {
  typedef Shape<W1, W2, W3> S;
  const int g = lane >> 4, n = lane & 15;
  const float *w1 = (const float *)(net + S::O_W1), *b1 = (const float *)(net + S::O_B1);
  const float *b2 = (const float *)(net + S::O_B2);
  float h1[2][4], hd1[2][4];
  layer1<W1, true>(w1, b1, s, g, h1, hd1);
  if constexpr (S::XL2)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      *(float4 *)(h1s + n * S::S1 + 16 * mt + 4 * g) = make_float4(h1[mt][0], h1[mt][1], h1[mt][2], h1[mt][3]);
      *(float4 *)(hd1s + n * S::S1 + 16 * mt + 4 * g) = make_float4(hd1[mt][0], hd1[mt][1], hd1[mt][2], hd1[mt][3]);
    }
  Split8<P> B2h[1] = {split8<P>(h1[0], h1[1])}, B2d[1] = {split8<P>(hd1[0], hd1[1])};
  v4f acc2[S::MT2], acc2d[S::MT2];
  layer_mfma<P, S::MT2, 1>(net + S::O_A2, b2, B2h, lane, g, acc2);
  layer_mfma_tan<P, S::MT2, 1>(net + S::O_A2, B2d, lane, acc2d);
  wsync();
#pragma unroll
  for (int mt = 0; mt < S::MT2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * mt + 4 * g + r;
      float hv = 0.f, dv = 0.f;
      if (16 * mt < W2 && f < W2) {
        const float th = tanh_f(acc2[mt][r]);
        hv = th + skip_val<W1, W2, S::SK2, 2>(f, mt, r, h1, h1s, n, S::S1);
        dv = (1.f - th * th) * acc2d[mt][r] + skip_val<W1, W2, S::SK2, 2>(f, mt, r, hd1, hd1s, n, S::S1);
      }
      h2[mt][r] = hv;
      hd2[mt][r] = dv;
    }
}

// M = W3 dT for one (atom, net) as split 16-bit halves MA (lane (g, n): row
// c = n < 4 of M^T, the layer-3 inputs in the permuted K order; rows n >= 4
// are zero) and q = b3^T dT (q[c] in every lane).  dT (rows dtr, from
// dt_rows) is staged in the wave's scratch dTs first; on return every lane
// is done with it.
// dT rows lane and lane + 64 of atom i (zero past M1), as lin_m_q stages
// them; unconditional loads, masked after
__device__ inline void dt_rows(const MixArgs &a, int i, int lane, float4 (&dtr)[2]) {
  const int M1 = a.d.M1;
  const float4 *dTi = (const float4 *)a.dT32 + (int64_t)i * M1;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int r = lane + 64 * m;
    const float4 v = dTi[r < M1 ? r : M1 - 1];
    const float k = r < M1 ? 1.f : 0.f;
    dtr[m] = make_float4(v.x * k, v.y * k, v.z * k, v.w * k);
  }
}

template <int W1, int W2, int W3, int P>
__device__ inline void lin_m_q(const float4 (&dtr)[2], const unsigned char *a3b, const float *b3, float *dTs, int lane,
                               Split8<P> &MA, float (&q)[4]) {
  typedef LinShape<W1, W2, W3> LS;
  typedef typename HT<P>::v8 V;
  static_assert(LS::DT_ROWS == 128, "dT is staged as two rows per lane");
  const int g = lane >> 4, n = lane & 15;
  ((float4 *)dTs)[lane] = dtr[0];
  ((float4 *)dTs)[lane + 64] = dtr[1];
  wsync();
  // B operands of W3 dT (K = outputs f = 32 kk + 8 g + v, N = components
  // c = n); lanes n >= 4 take zeros: their loads read component n & 3 and
  // are scaled by 0
  const float nmask = n < 4 ? 1.f : 0.f;
  v4f Macc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
  for (int kk = 0; kk < LS::KF; ++kk) {
    float x[4], y[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // rows f >= M1 of dTs are zero
      const int f0 = 32 * kk + 8 * g + v, f1 = f0 + 4;
      x[v] = dTs[4 * f0 + (n & 3)] * nmask;
      y[v] = dTs[4 * f1 + (n & 3)] * nmask;
    }
    const Split8<P> dB = split8<P>(x, y);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const V av = *(const V *)(a3b + ((mt * LS::KF + kk) * 64 + lane) * 16);
      Macc[mt] = mfma16<P>(av, dB.hi, Macc[mt]);
      Macc[mt] = mfma16<P>(av, dB.lo, Macc[mt]);
    }
  }
  // q: lane takes the entries lane + 64 m of the [M1][4] block (component
  // lane & 3), then the lanes of one component are summed
  float qv = 0.f;
  for (int o = lane; o < W3 * 4; o += 64) qv += b3[o >> 2] * dTs[o];
  qv += __shfl_xor(qv, 4);
  qv += __shfl_xor(qv, 8);
  qv += __shfl_xor(qv, 16);
  qv += __shfl_xor(qv, 32);
#pragma unroll
  for (int c = 0; c < 4; ++c) q[c] = __shfl(qv, c);
  float mx[4], my[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mx[r] = Macc[0][r];
    my[r] = Macc[1][r];
  }
  MA = split8<P>(mx, my);
  wsync();
}

// Projected table of one (atom, net) into the wave's scratch pts:
// P[row][c] = sum_f coef[row][f] M[f][c], plus q[c] on the rows of h2 itself,
// as PT_TILES MFMA tiles of 16 rows (A = M^T split, B = the coefficient image
// in its hi and lo halves, loaded a tile ahead).  Output lane (0, n) holds
// row 16 tt + n for the four components.  The tile loop stays a loop (two
// tiles per trip): unrolled, the product chains of all tiles were scheduled
// side by side and their accumulators spilled.
template <int P>
__device__ inline void proj_build(const unsigned char *img, const Split8<P> &MA, const float (&q)[4], float *pts,
                                  int lane) {
  typedef typename HT<P>::v8 V;
  const int g = lane >> 4, n = lane & 15;
  V bh = *(const V *)(img + 16 * lane), bl = *(const V *)(img + 1024 + 16 * lane);
#pragma unroll 2
  for (int tt = 0; tt < PT_TILES; ++tt) {
    const int tn = tt + 1 < PT_TILES ? tt + 1 : tt;
    const V nh = *(const V *)(img + (2 * tn) * 1024 + 16 * lane);
    const V nl = *(const V *)(img + (2 * tn + 1) * 1024 + 16 * lane);
    const int row = 16 * tt + n;
    const float qs = (row % 3 == 0) ? 1.f : 0.f;
    v4f acc = v4f{q[0] * qs, q[1] * qs, q[2] * qs, q[3] * qs};
    acc = mfma16<P>(MA.hi, bh, acc);
    acc = mfma16<P>(MA.hi, bl, acc);
    acc = mfma16<P>(MA.lo, bh, acc);
    if (g == 0) *(float4 *)(pts + 4 * row) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    bh = nh;
    bl = nl;
  }
  wsync();
}

// dE/dR of one neighbour from the projected table: cubic Hermite in the
// interval k of s, a = M^T h2(s) + q, b = M^T dh2/ds(s), and
// dE/dR = a + (R . b) e_0
__device__ inline float4 proj_eval(const float *pts, float4 r4, float inv_ds) {
  const float x = r4.x * inv_ds;
  int k = (int)x;
  k = k < TAB_K - 1 ? k : TAB_K - 1;
  const float t = x - (float)k, t2 = t * t, t3 = t2 * t;
  const float h10 = t3 - 2.f * t2 + t, h01 = 3.f * t2 - 2.f * t3, h11 = t3 - t2;
  const float e01 = 6.f * (t - t2), e10 = 3.f * t2 - 4.f * t + 1.f, e11 = 3.f * t2 - 2.f * t;
  const float4 *pk = (const float4 *)pts + 3 * k;
  const float4 py = pk[0], pdy = pk[1], pm0 = pk[2], pm1 = pk[5];
  const float a0 = h01 * pdy.x + h10 * pm0.x + h11 * pm1.x + py.x;
  const float a1 = h01 * pdy.y + h10 * pm0.y + h11 * pm1.y + py.y;
  const float a2 = h01 * pdy.z + h10 * pm0.z + h11 * pm1.z + py.z;
  const float a3 = h01 * pdy.w + h10 * pm0.w + h11 * pm1.w + py.w;
  const float b0 = e01 * pdy.x + e10 * pm0.x + e11 * pm1.x;
  const float b1 = e01 * pdy.y + e10 * pm0.y + e11 * pm1.y;
  const float b2 = e01 * pdy.z + e10 * pm0.z + e11 * pm1.z;
  const float b3 = e01 * pdy.w + e10 * pm0.w + e11 * pm1.w;
  const float bd = (r4.x * b0 + r4.y * b1 + r4.z * b2 + r4.w * b3) * inv_ds;
  return make_float4(a0 + bd, a1, a2, a3);
}

// FP64 force of the pair (i, slot) from gr = dE/dR, with the neighbour's
// share to the block's LDS accumulator (CELL, when its cell is held) or to
// global memory
// (D4 = displacement and r^2 of the pair, slot = the neighbour's LDS slot
// or -1)
template <bool CELL>
__device__ inline void scatter_pair(const MixArgs &a, const CellCtx &cc, int64_t slot_idx, const double4 &D4, int j,
                                    int slot, float4 gr, double rc, double rcs, double inv_w, double &fi0,
                                    double &fi1, double &fi2, double (&vir)[9]) {
  double gx, gy, gz;
  pair_force(D4, gr, rc, rcs, inv_w, gx, gy, gz, fi0, fi1, fi2, vir);
  if (a.net_deriv) {
    double *nd = a.net_deriv + slot_idx * 4;
    nd[0] = gr.x; nd[1] = gr.y; nd[2] = gr.z; nd[3] = gr.w;
  }
  if (slot >= 0) {
    lds_add(cc.facc + 3 * slot + 0, -gx);
    lds_add(cc.facc + 3 * slot + 1, -gy);
    lds_add(cc.facc + 3 * slot + 2, -gz);
  } else {
    unsafeAtomicAdd(a.force + 3 * (int64_t)j + 0, -gx);
    unsafeAtomicAdd(a.force + 3 * (int64_t)j + 1, -gy);
    unsafeAtomicAdd(a.force + 3 * (int64_t)j + 2, -gz);
  }
}

// F_i: wave sum, one add per component (to the LDS accumulator when the
// atom's own slot is held)
template <bool CELL>
__device__ inline void store_fi(const MixArgs &a, const CellCtx &cc, int i, int li, int lane, double fi0, double fi1,
                                double fi2) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    fi0 += __shfl_xor(fi0, o);
    fi1 += __shfl_xor(fi1, o);
    fi2 += __shfl_xor(fi2, o);
  }
  if (lane == 0) {
    if (CELL && li < cc.cap) {
      double *f = cc.facc + 3 * (13 * cc.cap + li);
      lds_add(f + 0, fi0);
      lds_add(f + 1, fi1);
      lds_add(f + 2, fi2);
    } else {
      unsafeAtomicAdd(a.force + 3 * (int64_t)i + 0, fi0);
      unsafeAtomicAdd(a.force + 3 * (int64_t)i + 1, fi1);
      unsafeAtomicAdd(a.force + 3 * (int64_t)i + 2, fi2);
    }
  }
}

// backward of one (atom i, neighbour type u) with an affine-last-layer net,
// layers evaluated per neighbour: dE/dR per neighbour, the FP64 pair forces,
// F_i (into fi) and the virial.  CELL: neighbour forces go to the block's
// LDS accumulator when their cell is held, else straight to global memory
// with atomics.
template <int W1, int W2, int W3, int P, bool CELL>
__device__ inline void lin_bwd_net(const MixArgs &a, int i, int u, const unsigned char *smem, float *h1s, float *hd1s,
                                   float *dTs, float *gRs, int lane, double (&vir)[9], const CellCtx &cc,
                                   double &fi0, double &fi1, double &fi2) {
  typedef Shape<W1, W2, W3> S;
  typedef LinShape<W1, W2, W3> LS;
  const Dims &d = a.d;
  const int g = lane >> 4, n = lane & 15;
  const double rc = d.rcut, rcs = d.rcut_smth, inv_w = 1.0 / (d.rcut - d.rcut_smth);
  const double4 xi = a.xw[i];
  const int t = (int)xi.w;
  const unsigned char *net = smem + (t * d.ntypes + u) * LS::NET_BYTES;
  const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
  if (cnt == 0) return;
  const int64_t base = (int64_t)i * d.nnei + d.off[u];
  // M and q are rebuilt per net so that they hold no registers across nets
  Split8<P> MA;
  float q[4];
  float4 dtr[2];
  dt_rows(a, i, lane, dtr);
  lin_m_q<W1, W2, W3, P>(dtr, net + LS::O_A3B, (const float *)(net + S::O_B3), dTs, lane, MA, q);
  float4 r4n = rt_row(a.rt, base, n, cnt);
  // force-pass operands of the current 64-neighbour chunk, loaded a chunk ahead
  double4 pjc = xi;  // neighbour positions of the chunk, gathered at its first tile
  int jc = a.nlist[base + (lane < cnt ? lane : cnt - 1)];
  uint32_t codec = 0;
  for (int n0 = 0; n0 < cnt; n0 += 16) {
    // this tile's environment rows; the next tile's are loaded meanwhile
    const float4 r4 = r4n;
    if (n0 + 16 < cnt) r4n = rt_row(a.rt, base, n0 + 16 + n, cnt);
    float h2[S::MT2][4], hd2[S::MT2][4];
    layers_h2<W1, W2, W3, P>(net, r4.x, lane, h1s, hd1s, h2, hd2);
    const Split8<P> B3h = split8<P>(h2[0], h2[1]), B3d = split8<P>(hd2[0], hd2[1]);
    // a = M^T h2 and b = M^T dh2/ds (lane (g, n): component c = 4 g + r of neighbour n)
    v4f ca = v4f{0.f, 0.f, 0.f, 0.f}, cb = v4f{0.f, 0.f, 0.f, 0.f};
    ca = mfma16<P>(MA.hi, B3h.hi, ca);
    ca = mfma16<P>(MA.hi, B3h.lo, ca);
    ca = mfma16<P>(MA.lo, B3h.hi, ca);
    cb = mfma16<P>(MA.hi, B3d.hi, cb);
    cb = mfma16<P>(MA.hi, B3d.lo, cb);
    cb = mfma16<P>(MA.lo, B3d.hi, cb);
    const int slot0 = n0 & 63;
    if (g == 0) {
      // dE/dR = a + q + (R . b) e_0
      const float bd = r4.x * cb[0] + r4.y * cb[1] + r4.z * cb[2] + r4.w * cb[3];
      *(float4 *)(gRs + 4 * (slot0 + n)) = make_float4(ca[0] + q[0] + bd, ca[1] + q[1], ca[2] + q[2], ca[3] + q[3]);
    }
    // positions and cell codes of this chunk's neighbours (jc arrived during the tile)
    if (slot0 == 0) {
      pjc = a.xw[jc];
      if (CELL) codec = cc.code[jc];
    }
    wsync();
    // every 64 neighbours (or at the end of the type block): FP64 force pass
    if (((n0 + 16) & 63) == 0 || n0 + 16 >= cnt) {
      const int c0 = n0 & ~63;
      const int qq = c0 + lane;
      if (qq < cnt) {
        const float4 gr = *(const float4 *)(gRs + 4 * lane);
        scatter_pair<CELL>(a, cc, base + qq, pair_disp_sq(xi, pjc, a.L[0], a.L[1], a.L[2]), jc,
                           CELL ? cell_slot(cc, codec) : -1, gr, rc, rcs, inv_w, fi0, fi1, fi2, vir);
      }
      if (c0 + 64 < cnt) jc = a.nlist[base + (qq + 64 < cnt ? qq + 64 : cnt - 1)];
      wsync();
    }
  }
}

// backward of one atom i, layers evaluated per neighbour (li = index of i in
// its cell, CELL only)
template <int W1, int W2, int W3, int P, bool CELL>
__device__ inline void lin_bwd_atom(const MixArgs &a, int i, const unsigned char *smem, float *h1s, float *hd1s,
                                    float *dTs, float *gRs, int lane, double (&vir)[9], const CellCtx &cc, int li) {
  double fi0 = 0.0, fi1 = 0.0, fi2 = 0.0;
  for (int u = 0; u < a.d.ntypes; ++u)
    lin_bwd_net<W1, W2, W3, P, CELL>(a, i, u, smem, h1s, hd1s, dTs, gRs, lane, vir, cc, fi0, fi1, fi2);
  store_fi<CELL>(a, cc, i, li, lane, fi0, fi1, fi2);
}

// The same with the student table, by projection: per (atom, net) the table
// is contracted with M = W3 dT once (proj_build), then every neighbour takes
// one lane and interpolates 3 x 4 projected values (proj_eval).  The list is
// sorted by distance, so the nearest neighbour (slot 0) has the largest s of
// the net's block up to ties of the quantised distance (1e-8 A); a net whose
// slot 0 comes within 1e-6 (relative) of the table's end is appended to the
// deferred list instead, for k_embed_bwd_defer to evaluate with the layers.
// nb: the per-net LDS images (stride nb_bytes; W3 dT operands at o_a3b, b3
// at o_b3), img: the projection images (stride PIMG_BYTES, LDS or global),
// pts: the wave's PT_BYTES of scratch.
// dtr: atom i's dT rows (dt_rows) on entry, the rows of atom inext (>= 0)
// on return, loaded while i is evaluated.
template <int W1, int W2, int W3, int P, bool CELL>
__device__ inline void lin_bwd_atom_proj(const MixArgs &a, int i, int inext, float4 (&dtr)[2], const unsigned char *nb,
                                         int nb_bytes, int o_a3b, int o_b3, const unsigned char *img, float *pts,
                                         int lane, double (&vir)[9], const CellCtx &cc, int li) {
  const Dims &d = a.d;
  const double rc = d.rcut, rcs = d.rcut_smth, inv_w = 1.0 / (d.rcut - d.rcut_smth);
  const double4 xi = a.xw[i];
  const int t = (int)xi.w;
  double fi0 = 0.0, fi1 = 0.0, fi2 = 0.0;
  for (int u = 0; u < d.ntypes; ++u) {
    const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
    if (cnt == 0) continue;
    const int64_t base = (int64_t)i * d.nnei + d.off[u];
    // slot data of the first chunk and the neighbours of the second, in
    // flight during the table build
    float4 r4 = rt_row_m(a.rt, base, lane, cnt);
    int jc = a.nlist[base + (lane < cnt ? lane : cnt - 1)];
    int jn = a.nlist[base + (lane + 64 < cnt ? lane + 64 : cnt - 1)];
    if (__shfl(r4.x, 0) * 1.000001f > a.tab_shi) {
      if (lane == 0) a.defer[atomicAdd(a.defer_count, 1u)] = i * d.ntypes + u;
      continue;
    }
    const int net_id = t * d.ntypes + u;
    const unsigned char *net = nb + (size_t)net_id * nb_bytes;
    Split8<P> MA;
    float q[4];
    lin_m_q<W1, W2, W3, P>(dtr, net + o_a3b, (const float *)(net + o_b3), pts, lane, MA, q);
    if (u == d.ntypes - 1 && inext >= 0) {
      dt_rows(a, inext, lane, dtr);
      inext = -1;
    }
    proj_build<P>(img + (size_t)net_id * PIMG_BYTES, MA, q, pts, lane);
    uint32_t codec = CELL ? cc.code[jc] : 0u;
    double4 pjc = pos3(a.xw, jc);
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const int qq = c0 + lane;
      // everything that reads this chunk's loads (issued during the chunk
      // before) comes first: a read after the next loads would make the
      // compiler wait for those too, as it cannot count the force pass's
      // conditional stores in between
      const double4 D4 = pair_disp_sq(xi, pjc, a.L[0], a.L[1], a.L[2]);
      const int slot = CELL ? cell_slot(cc, codec) : -1;
      const float4 gr = proj_eval(pts, r4, a.tab_inv_ds);
      __builtin_amdgcn_sched_barrier(0);
      // loads for the next chunks (unconditional: past the block the last
      // real slot is reread): the neighbours of the one after next, this
      // one's successor's cell codes and positions (its neighbours arrived
      // during the chunk before) and rows
      const int jnn = a.nlist[base + (qq + 128 < cnt ? qq + 128 : cnt - 1)];
      const uint32_t coden = CELL ? cc.code[jn] : 0u;
      const double4 pjn = pos3(a.xw, jn);
      const float4 r4n = rt_row_m(a.rt, base, qq + 64, cnt);
      if (qq < cnt) scatter_pair<CELL>(a, cc, base + qq, D4, jc, slot, gr, rc, rcs, inv_w, fi0, fi1, fi2, vir);
      r4 = r4n;
      jc = jn;
      jn = jnn;
      pjc = pjn;
      codec = coden;
    }
    wsync();  // every lane is done with the table before the next net overwrites it
  }
  if (inext >= 0) dt_rows(a, inext, lane, dtr);  // the last net had no neighbours or was deferred
  store_fi<CELL>(a, cc, i, li, lane, fi0, fi1, fi2);
}

template <int W1, int W2, int W3, int P, bool PROJ>
__global__ void __launch_bounds__(64 * MIX_WAVES, 3) k_embed_bwd_lin(MixArgs a) {
  typedef LinShape<W1, W2, W3> LS;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double vred[MIX_WAVES][9];
  const int nnets = a.d.ntypes * a.d.ntypes;
  copy_nets(smem, a.nets, nnets * LS::NET_BYTES);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned char *ws = smem + nnets * LS::NET_BYTES + wv * LS::P2_BYTES;
  float *h1s = (float *)(ws + LS::P2_H1), *hd1s = h1s + 16 * Shape<W1, W2, W3>::S1;
  float *dTs = (float *)(ws + LS::P2_DT);
  float *gRs = (float *)(ws + LS::P2_GR);
  double vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0;
  const CellCtx cc{};
  int64_t p0, p1;
  wave_rows(a.rows, p0, p1);
  for (int64_t p = p0; p < p1; ++p) {
    const int i = a.atom_of_pos[p];
    if (i < 0) continue;
    if constexpr (PROJ) {
      float4 dtr[2];
      dt_rows(a, i, lane, dtr);
      lin_bwd_atom_proj<W1, W2, W3, P, false>(a, i, -1, dtr, smem, LS::NET_BYTES, LS::O_A3B, Shape<W1, W2, W3>::O_B3,
                                              a.pimg, (float *)ws, lane, vir, cc, 0);
    }
    else lin_bwd_atom<W1, W2, W3, P, false>(a, i, smem, h1s, hd1s, dTs, gRs, lane, vir, cc, 0);
  }
  finish_block_virial(a, vir, vred, lane, wv);
}

// The nets the table kernels deferred (a neighbour beyond the table's
// range), by the layers: wave w of the grid takes entries w, w + waves, ...
// of the list (i ntypes + u), forces by global atomics, the block's virial
// partial in vir_part[blockIdx] (the host offsets vir_part past the main
// kernel's partials).  With an empty list the blocks write zero partials.
template <int W1, int W2, int W3, int P>
__global__ void __launch_bounds__(64 * MIX_WAVES, 3) k_embed_bwd_defer(MixArgs a) {
  typedef LinShape<W1, W2, W3> LS;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double vred[MIX_WAVES][9];
  const uint32_t cnt = *a.defer_count;
  if (cnt == 0) {  // uniform over the grid
    if (threadIdx.x < 9) a.vir_part[(int64_t)blockIdx.x * 9 + threadIdx.x] = 0.0;
    return;
  }
  const int nnets = a.d.ntypes * a.d.ntypes;
  copy_nets(smem, a.nets, nnets * LS::NET_BYTES);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned char *ws = smem + nnets * LS::NET_BYTES + wv * LS::P2_BYTES;
  float *h1s = (float *)(ws + LS::P2_H1), *hd1s = h1s + 16 * Shape<W1, W2, W3>::S1;
  float *dTs = (float *)(ws + LS::P2_DT);
  float *gRs = (float *)(ws + LS::P2_GR);
  double vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0;
  const CellCtx cc{};
  const uint32_t nwaves = gridDim.x * MIX_WAVES;
  for (uint32_t e = blockIdx.x * MIX_WAVES + wv; e < cnt; e += nwaves) {
    const int code = a.defer[e];
    const int i = code / a.d.ntypes, u = code % a.d.ntypes;
    double fi0 = 0.0, fi1 = 0.0, fi2 = 0.0;
    lin_bwd_net<W1, W2, W3, P, false>(a, i, u, smem, h1s, hd1s, dTs, gRs, lane, vir, cc, fi0, fi1, fi2);
    store_fi<false>(a, cc, i, 0, lane, fi0, fi1, fi2);
  }
  finish_block_virial(a, vir, vred, lane, wv);
}

// Cell-ordered backward (affine-last-layer nets): block b takes cells b,
// b + grid, ... of the list grid (side >= the list radius, >= 3 cells per
// axis, so every neighbour of a cell's atoms lies in the 27 cells around it).
// The waves take the cell's atoms in turn; every pair force lands in the LDS
// accumulator, which is then copied to part[26 - s][position][3] for the 27
// neighbour cells (s = offset of the destination cell seen from this one,
// 26 - s = this cell seen from the destination).  Each part entry is written
// by exactly one cell, so no global atomics are needed; k_cell_gather adds
// the 27 parts of every atom.  Atoms past the capacity use global atomics.
// With the table (PROJ) the block holds per net only b3 and the W3 dT
// operands (the tail of the net image from O_B3 on) and, after them, the
// nets' projection images, so the table build reads LDS, not L2.
template <int W1, int W2, int W3>
struct CellShape {
  typedef Shape<W1, W2, W3> S;
  typedef LinShape<W1, W2, W3> LS;
  static_assert(!S::XL2, "the cell kernel keeps no cross-lane skip scratch");
  static constexpr int W_DT = 0;                        // float [DT_ROWS][4]
  static constexpr int W_GR = LS::DT_ROWS * 16;         // float [64][4]
  // per wave: dT and gR (layers), or the projected table (dT staged in it first)
  static constexpr int W_BYTES = W_GR + 1024 > PT_BYTES ? W_GR + 1024 : PT_BYTES;
  static constexpr int NB = LS::NET_BYTES - S::O_B3;   // per-net bytes kept with the table
  static_assert(S::O_B3 % 16 == 0 && NB % 16 == 0, "16-byte copies");
  static constexpr size_t fixed(int nnets, bool proj) {
    return proj ? (size_t)nnets * (NB + PIMG_BYTES) : (size_t)nnets * LS::NET_BYTES;
  }
};

template <int W1, int W2, int W3, int P, bool PROJ>
__global__ void __launch_bounds__(64 * cell_waves(PROJ), 1) k_embed_bwd_cells(MixArgs a, CellArgs ca) {
  typedef LinShape<W1, W2, W3> LS;
  typedef CellShape<W1, W2, W3> CS;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double vred[CELL_WAVES][9];
  const int nnets = a.d.ntypes * a.d.ntypes;
  const int nw = blockDim.x >> 6;
  if constexpr (PROJ) {
    for (int k = 0; k < nnets; ++k)
      copy_nets(smem + k * CS::NB, a.nets + (size_t)k * LS::NET_BYTES + Shape<W1, W2, W3>::O_B3, CS::NB);
    copy_nets(smem + nnets * CS::NB, a.pimg, nnets * PIMG_BYTES);
  } else {
    copy_nets(smem, a.nets, nnets * LS::NET_BYTES);
  }
  const size_t fixed = CS::fixed(nnets, PROJ);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned char *ws = smem + fixed + wv * CS::W_BYTES;
  float *dTs = (float *)(ws + CS::W_DT);
  float *gRs = (float *)(ws + CS::W_GR);
  double *facc = (double *)(smem + fixed + nw * CS::W_BYTES);
  const int nacc = 27 * 3 * ca.cap;
  double vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0;
  for (int64_t c = blockIdx.x; c < ca.ncell; c += gridDim.x) {
    for (int o = threadIdx.x; o < nacc; o += blockDim.x) facc[o] = 0.0;
    __syncthreads();
    CellCtx cc;
    cc.facc = facc;
    cc.code = ca.code;
    cc.nc0 = ca.nc[0];
    cc.nc1 = ca.nc[1];
    cc.nc2 = ca.nc[2];
    cc.cap = ca.cap;
    // uniform over the block: kept in scalar registers
    cc.cz = __builtin_amdgcn_readfirstlane((int)(c % cc.nc2));
    cc.cy = __builtin_amdgcn_readfirstlane((int)((c / cc.nc2) % cc.nc1));
    cc.cx = __builtin_amdgcn_readfirstlane((int)(c / ((int64_t)cc.nc1 * cc.nc2)));
    const int b = ca.cell_start[c], e = ca.cell_start[c + 1];
    float4 dtr[2];  // table path: dT of the wave's next atom, loaded during the one before
    if (PROJ && b + wv < e) dt_rows(a, ca.cell_atoms[b + wv], lane, dtr);
    for (int k = b + wv; k < e; k += nw) {
      if constexpr (PROJ)
        lin_bwd_atom_proj<W1, W2, W3, P, true>(a, ca.cell_atoms[k], k + nw < e ? ca.cell_atoms[k + nw] : -1, dtr, smem,
                                               CS::NB, LS::O_A3B - Shape<W1, W2, W3>::O_B3, 0,
                                               smem + nnets * CS::NB, (float *)ws, lane, vir, cc, k - b);
      else
        lin_bwd_atom<W1, W2, W3, P, true>(a, ca.cell_atoms[k], smem, nullptr, nullptr, dTs, gRs, lane, vir, cc,
                                          k - b);
    }
    __syncthreads();
    for (int s = 0; s < 27; ++s) {
      const int x = (cc.cx + s / 9 - 1 + cc.nc0) % cc.nc0, y = (cc.cy + (s / 3) % 3 - 1 + cc.nc1) % cc.nc1,
                z = (cc.cz + s % 3 - 1 + cc.nc2) % cc.nc2;
      const int64_t c2 = ((int64_t)x * cc.nc1 + y) * cc.nc2 + z;
      const int b2 = ca.cell_start[c2], m2 = min(ca.cell_start[c2 + 1] - b2, ca.cap);
      double *dst = ca.part + ((int64_t)(26 - s) * ca.n + b2) * 3;
      const double *src = facc + 3 * s * ca.cap;
      for (int o = threadIdx.x; o < 3 * m2; o += blockDim.x) dst[o] = src[o];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double v = vir[k];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    if (lane == 0) vred[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += vred[w][threadIdx.x];
    a.vir_part[(int64_t)blockIdx.x * 9 + threadIdx.x] = v;
  }
}

// F[j] += the 27 parts of the atom at cell-ordered position p
__global__ void k_cell_gather(CellArgs ca, double *F) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ca.n) return;
  const int j = ca.cell_atoms[p];
  const int l = (int)(p - ca.cell_start[ca.cell_of[j]]);
  if (l >= ca.cap) return;
  double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll 9
  for (int s = 0; s < 27; ++s) {
    const double *q = ca.part + ((int64_t)s * ca.n + p) * 3;
    fx += q[0];
    fy += q[1];
    fz += q[2];
  }
  F[3 * (int64_t)j + 0] += fx;
  F[3 * (int64_t)j + 1] += fy;
  F[3 * (int64_t)j + 2] += fz;
}

// ---------------------------------------------------------------------------
// host side: weight packing and dispatch
// ---------------------------------------------------------------------------
template <int W1, int W2, int W3, int LIN>
static size_t net_bytes_t() {
  if constexpr (LIN) return LinShape<W1, W2, W3>::NET_BYTES;
  else return Shape<W1, W2, W3>::NET_BYTES;
}

static inline uint16_t to_f16(float x) {
  _Float16 h = (_Float16)x;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

static inline uint16_t to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}

// Pack one net (t,u) into the LDS image; W[l] are row-major [in][out] doubles.
template <int W1, int W2, int W3, int LIN>
static void pack_net_t(const double *const *W, const double *const *b, int prec, unsigned char *out) {
  typedef Shape<W1, W2, W3> S;
  std::memset(out, 0, net_bytes_t<W1, W2, W3, LIN>());
  float *w1 = (float *)(out + S::O_W1), *b1 = (float *)(out + S::O_B1);
  for (int f = 0; f < W1; ++f) {
    w1[f] = (float)W[0][f];
    b1[f] = (float)b[0][f];
  }
  auto h16 = [&](double v) { return prec == 0 ? to_f16((float)v) : to_bf16((float)v); };
  // permuted K slot of (kk, lane group g, element v)
  auto kslot = [](int kk, int g, int v) { return 16 * (2 * kk + v / 4) + 4 * g + (v % 4); };
  uint16_t *A2 = (uint16_t *)(out + S::O_A2);
  for (int mt = 0; mt < S::MT2; ++mt)
    for (int lane = 0; lane < 64; ++lane)
      for (int v = 0; v < 8; ++v) {
        const int fo = 16 * mt + (lane & 15), fi = kslot(0, lane >> 4, v);
        A2[((mt * 1 + 0) * 64 + lane) * 8 + v] = (fo < W2 && fi < W1) ? h16(W[1][fi * W2 + fo]) : 0;
      }
  float *b2 = (float *)(out + S::O_B2);
  for (int f = 0; f < W2; ++f) b2[f] = (float)b[1][f];
  uint16_t *A3 = (uint16_t *)(out + S::O_A3);
  for (int mt = 0; mt < S::MT3; ++mt)
    for (int kk = 0; kk < S::KS3; ++kk)
      for (int lane = 0; lane < 64; ++lane)
        for (int v = 0; v < 8; ++v) {
          const int fo = 16 * mt + (lane & 15), fi = kslot(kk, lane >> 4, v);
          A3[((mt * S::KS3 + kk) * 64 + lane) * 8 + v] = (fo < W3 && fi < W2) ? h16(W[2][fi * W3 + fo]) : 0;
        }
  float *b3 = (float *)(out + S::O_B3);
  for (int f = 0; f < W3; ++f) b3[f] = (float)b[2][f];
  if constexpr (LIN) {
    // W3 itself as A operands of M = W3 dT: rows k = 16 mt + lane%16,
    // K = outputs f = 32 kk + 8 (lane/16) + v in natural order
    typedef LinShape<W1, W2, W3> LS;
    uint16_t *A3B = (uint16_t *)(out + LS::O_A3B);
    for (int mt = 0; mt < 2; ++mt)
      for (int kk = 0; kk < LS::KF; ++kk)
        for (int lane = 0; lane < 64; ++lane)
          for (int v = 0; v < 8; ++v) {
            const int k = 16 * mt + (lane & 15), f = 32 * kk + 8 * (lane >> 4) + v;
            A3B[((mt * LS::KF + kk) * 64 + lane) * 8 + v] = (k < W2 && f < W3) ? h16(W[2][k * W3 + f]) : 0;
          }
  }
}

template <int W1, int W2, int W3, int LIN, int P>
static void launch_t(hipStream_t s, const MixArgs &a, int pass, int grid) {
  typedef Shape<W1, W2, W3> S;
  const int nnets = a.d.ntypes * a.d.ntypes;
  if constexpr (LIN) {
    typedef LinShape<W1, W2, W3> LS;
    const size_t tab = a.tab ? (size_t)nnets * TAB_BYTES : 0;
    if (pass == 1) {
      const size_t shm = (size_t)nnets * LS::NET_BYTES + tab + (size_t)MIX_WAVES * LS::P1_BYTES;
      hipLaunchKernelGGL((k_embed_fwd_lin<W1, W2, W3, P>), dim3(grid), dim3(64 * MIX_WAVES), shm, s, a);
    } else {
      // the backward takes the table through its projection image, not from LDS
      const size_t shm = (size_t)nnets * LS::NET_BYTES + (size_t)MIX_WAVES * LS::P2_BYTES;
      if (a.tab) hipLaunchKernelGGL((k_embed_bwd_lin<W1, W2, W3, P, true>), dim3(grid), dim3(64 * MIX_WAVES), shm, s, a);
      else hipLaunchKernelGGL((k_embed_bwd_lin<W1, W2, W3, P, false>), dim3(grid), dim3(64 * MIX_WAVES), shm, s, a);
    }
    return;
  }
  if (pass == 1) {
    const size_t shm = (size_t)nnets * S::NET_BYTES + (size_t)MIX_WAVES * S::P1_BYTES;
    hipLaunchKernelGGL((k_embed_fwd_mix<W1, W2, W3, LIN, P>), dim3(grid), dim3(64 * MIX_WAVES), shm, s, a);
  } else {
    const size_t shm = (size_t)nnets * S::NET_BYTES + (size_t)MIX_WAVES * S::P2_BYTES;
    hipLaunchKernelGGL((k_embed_bwd_mix<W1, W2, W3, LIN, P>), dim3(grid), dim3(64 * MIX_WAVES), shm, s, a);
  }
}

template <int W1, int W2, int W3, int LIN>
static size_t lds_t(int ntypes, int pass) {
  if constexpr (LIN) {
    typedef LinShape<W1, W2, W3> LS;
    return (size_t)ntypes * ntypes * LS::NET_BYTES + (size_t)MIX_WAVES * (pass == 1 ? LS::P1_BYTES : LS::P2_BYTES);
  } else {
    typedef Shape<W1, W2, W3> S;
    return (size_t)ntypes * ntypes * S::NET_BYTES + (size_t)MIX_WAVES * (pass == 1 ? S::P1_BYTES : S::P2_BYTES);
  }
}

// whether the affine-net kernels of a shape fit the LDS with the student table
template <int W1, int W2, int W3, int LIN>
static bool tab_fits_t(int ntypes) {
  if constexpr (LIN == 0 || Shape<W1, W2, W3>::XL2 || W2 != 32) {
    return false;
  } else {
    typedef LinShape<W1, W2, W3> LS;
    // the forward holds the table in LDS, the backward only the nets
    const size_t nets = (size_t)ntypes * ntypes;
    return nets * (LS::NET_BYTES + TAB_BYTES) + (size_t)MIX_WAVES * LS::P1_BYTES <= 163840 &&
           nets * LS::NET_BYTES + (size_t)MIX_WAVES * LS::P2_BYTES <= 163840;
  }
}

// supported embedding shapes: widths of the three layers, affine last layer
#define DPK_MIX_SHAPES(X) X(25, 50, 100, 0) X(16, 32, 100, 0) X(16, 32, 100, 1) X(32, 64, 128, 0)

int mix_shape_id(const Dims &d) {
  if (d.n_emb != 3) return -1;
  int id = 0;
#define X(a_, b_, c_, l_)                                                                  \
  if (d.ew[1] == a_ && d.ew[2] == b_ && d.ew[3] == c_ && (d.emb_lin != 0) == (l_ != 0)) return id; \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
  return -1;
}

bool mix_tab_fits(int shape, int ntypes) {
  int id = 0;
#define X(a_, b_, c_, l_)                                     \
  if (shape == id) return tab_fits_t<a_, b_, c_, l_>(ntypes); \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
  return false;
}

size_t mix_net_bytes(int shape) {
  int id = 0;
#define X(a_, b_, c_, l_)                                  \
  if (shape == id) return net_bytes_t<a_, b_, c_, l_>(); \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
  return 0;
}

size_t mix_lds_bytes(int shape, int ntypes, int pass) {
  int id = 0;
#define X(a_, b_, c_, l_)                                     \
  if (shape == id) return lds_t<a_, b_, c_, l_>(ntypes, pass); \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
  return 0;
}

void mix_pack_net(int shape, const double *const *W, const double *const *b, int prec, unsigned char *out) {
  int id = 0;
#define X(a_, b_, c_, l_)                           \
  if (shape == id) {                                \
    pack_net_t<a_, b_, c_, l_>(W, b, prec, out);    \
    return;                                         \
  }                                                 \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
}

int mix_grid(int64_t rows) {
  int64_t g = (rows + MIX_WAVES - 1) / MIX_WAVES;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

template <int W1, int W2, int W3, int LIN, int P>
static void launch_defer_t(hipStream_t s, const MixArgs &a) {
  if constexpr (LIN != 0) {
    typedef LinShape<W1, W2, W3> LS;
    const size_t shm = (size_t)a.d.ntypes * a.d.ntypes * LS::NET_BYTES + (size_t)MIX_WAVES * LS::P2_BYTES;
    hipLaunchKernelGGL((k_embed_bwd_defer<W1, W2, W3, P>), dim3(DEFER_GRID), dim3(64 * MIX_WAVES), shm, s, a);
  }
}

void launch_embed_defer(hipStream_t s, const MixArgs &a) {
  int id = 0;
#define X(a_, b_, c_, l_)                                                      \
  if (a.shape == id) {                                                         \
    if (a.prec == 0) launch_defer_t<a_, b_, c_, l_, 0>(s, a);                  \
    else launch_defer_t<a_, b_, c_, l_, 1>(s, a);                              \
    return;                                                                    \
  }                                                                            \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
}

void launch_embed_mix(hipStream_t s, const MixArgs &a, int pass, int grid) {
  int id = 0;
#define X(a_, b_, c_, l_)                                 \
  if (a.shape == id) {                                    \
    if (a.prec == 0) launch_t<a_, b_, c_, l_, 0>(s, a, pass, grid); \
    else launch_t<a_, b_, c_, l_, 1>(s, a, pass, grid);   \
    return;                                               \
  }                                                       \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
}

// ---------------------------------------------------------------------------
// student table: the second layer of an affine-last-layer net, h2(s) and
// dh2/ds, is a function of the scalar s alone, so it is tabulated once per
// installed student on s_k = k ds (k = 0..TAB_K) in FP64 with the weights
// the kernels hold (layer 1 in FP32, W2 rounded to 16 bits) and interpolated
// per neighbour by cubic Hermite polynomials (the idea of tabulating the
// embedding net of a trained Deep Potential: Lu et al., J. Chem. Theory
// Comput. 18, 5559 (2022)).  Interpolation error of h2 ~ ds^4 max|h2^(4)| / 384.
// ---------------------------------------------------------------------------
__device__ inline double round16_dev(double v, int prec) {
  const float x = (float)v;
  if (prec == 0) return (double)(float)(_Float16)x;
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  return (double)__builtin_bit_cast(float, u);
}

__global__ void k_student_table(Dims d, EmbOffsets eo, const double *__restrict__ ew, int prec, double ds,
                                float *__restrict__ tab) {
  const int net = blockIdx.y;
  const int t = net / d.ntypes, u = net % d.ntypes;
  const int W1 = d.ew[1], W2 = d.ew[2];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (TAB_K + 1) * W2) return;
  const int k = idx / W2, f = idx % W2;
  const double sv = k * ds;
  const double *W0 = ew + eo.w[t][u][0], *b0 = ew + eo.b[t][u][0];
  const double *Wl = ew + eo.w[t][u][1], *bl = ew + eo.b[t][u][1];
  const int mp = d.emp[2];
  double z = (double)(float)bl[f], dz = 0.0, hs = 0.0, dhs = 0.0;
  for (int i = 0; i < W1; ++i) {
    const double w = (double)(float)W0[i], b = (double)(float)b0[i];
    const double h = tanh64(sv * w + b), dh = (1.0 - h * h) * w;
    const double wq = round16_dev(Wl[(size_t)i * mp + f], prec);
    z += wq * h;
    dz += wq * dh;
    if (i == f % W1) {
      hs = h;
      dhs = dh;
    }
  }
  const double th = tanh64(z);
  double y = th, dy = (1.0 - th * th) * dz;
  if (W2 == W1 || W2 == 2 * W1) {  // identity / doubling skip
    y += hs;
    dy += dhs;
  }
  float *row = tab + ((int64_t)net * (TAB_K + 1) + k) * TAB_STRIDE;
  row[2 * f] = (float)y;
  row[2 * f + 1] = (float)(ds * dy);
}

void launch_student_table(hipStream_t s, const Dims &d, const EmbOffsets &eo, const double *ew, int prec, double shi,
                          float *tab) {
  const int nets = d.ntypes * d.ntypes, n = (TAB_K + 1) * d.ew[2];
  hipLaunchKernelGGL(k_student_table, dim3((n + 127) / 128, nets), dim3(128), 0, s, d, eo, ew, prec, shi / TAB_K, tab);
}

// Operand image of the projected table (the backward's proj_build): per net
// PT_TILES blocks of 16 rows, row 3k + j of node k = (y_k, y_{k+1} - y_k, m_k)
// with y = h2(s_k) and m = ds dh2/ds(s_k) (the difference taken in FP32 from
// the table's values, y_{81} - y_{80} = 0), rows past 3 (TAB_K + 1) zero;
// B-operand lane (g, n) of tile tt holds row 16 tt + n at the layer-3 inputs
// f = 16 (v / 4) + 4 g + v % 4 (v = 0..7, the permuted K order of M),
// as hi = rn16(x) in one 1 KB block and lo = rn16(x - hi) in the next.
__global__ void k_student_pimg(int nets, const float *__restrict__ tab, int prec, unsigned char *__restrict__ img) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nets * PT_TILES * 512) return;
  const int v = idx & 7, lane = (idx >> 3) & 63, tt = (idx >> 9) % PT_TILES, net = idx / (PT_TILES * 512);
  const int row = 16 * tt + (lane & 15), f = 16 * (v >> 2) + 4 * (lane >> 4) + (v & 3);
  const int k = row / 3, j = row % 3;
  float x = 0.f;
  if (k <= TAB_K) {
    const float *r0 = tab + ((int64_t)net * (TAB_K + 1) + k) * TAB_STRIDE;
    if (j == 0) x = r0[2 * f];
    else if (j == 1) x = k < TAB_K ? r0[TAB_STRIDE + 2 * f] - r0[2 * f] : 0.f;
    else x = r0[2 * f + 1];
  }
  uint16_t *o = (uint16_t *)(img + (size_t)((net * PT_TILES + tt) * 2) * 1024) + lane * 8 + v;
  if (prec == 0) {
    const _Float16 h = (_Float16)x, l = (_Float16)(x - (float)h);
    o[0] = __builtin_bit_cast(uint16_t, h);
    o[512] = __builtin_bit_cast(uint16_t, l);
  } else {
    const __bf16 h = (__bf16)x, l = (__bf16)(x - (float)h);
    o[0] = __builtin_bit_cast(uint16_t, h);
    o[512] = __builtin_bit_cast(uint16_t, l);
  }
}

void launch_student_pimg(hipStream_t s, int nets, const float *tab, int prec, unsigned char *img) {
  const int n = nets * PT_TILES * 512;
  hipLaunchKernelGGL(k_student_pimg, dim3((n + 255) / 256), dim3(256), 0, s, nets, tab, prec, img);
}

// per atom the first real slot of each type block is its nearest neighbour
// of that type (the list is distance-sorted), so the largest s is the
// largest s of those slots; s >= 0, so its float bits order as unsigned
__global__ void k_smax(int64_t n, Dims d, const int32_t *__restrict__ nreal, const float4 *__restrict__ rt,
                       uint32_t *smax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.f;
  if (i < n)
    for (int u = 0; u < d.ntypes; ++u)
      if (nreal[i * d.ntypes + u] > 0) m = fmaxf(m, rt[i * d.nnei + d.off[u]].x);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(smax, __builtin_bit_cast(uint32_t, m));
}

void launch_smax(hipStream_t s, int64_t n, const Dims &d, const int32_t *nreal, const float4 *rt, uint32_t *smax) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_smax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, d, nreal, rt, smax);
}

// ---------------------------------------------------------------------------
// cell-ordered backward: configuration and launch
// ---------------------------------------------------------------------------
constexpr size_t CELL_LDS_MAX = 160 * 1024;  // LDS of one CU

template <int W1, int W2, int W3, int LIN>
static bool cells_config_t(int nnets, bool proj, int want, int need, int *cap, int *threads, size_t *lds) {
  if constexpr (LIN == 0 || Shape<W1, W2, W3>::XL2) {
    return false;
  } else {
    // the most waves whose scratch leaves room for an accumulator of at
    // least `need` atoms per cell; the accumulator then takes what is left,
    // up to `want`
    const size_t fixed = CellShape<W1, W2, W3>::fixed(nnets, proj);
    const size_t budget = CELL_LDS_MAX - sizeof(double) * CELL_WAVES * 9;
    const size_t per_atom = (size_t)27 * 3 * sizeof(double);
    for (int nw = cell_waves(proj); nw >= 4; nw -= 4) {
      const size_t b = fixed + (size_t)nw * CellShape<W1, W2, W3>::W_BYTES;
      if (b >= budget) continue;
      const int fit = (int)std::min<size_t>((budget - b) / per_atom, 255);
      if (fit < need) continue;
      *cap = std::min(want, fit);
      *threads = 64 * nw;
      *lds = b + (size_t)*cap * per_atom;
      return true;
    }
    return false;
  }
}

template <int W1, int W2, int W3, int LIN, int P>
static void launch_cells_t(hipStream_t s, const MixArgs &a, const CellArgs &ca, int grid, int threads, size_t lds) {
  if constexpr (LIN != 0 && !Shape<W1, W2, W3>::XL2) {
    if (a.tab) {
      (void)hipFuncSetAttribute((const void *)k_embed_bwd_cells<W1, W2, W3, P, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_embed_bwd_cells<W1, W2, W3, P, true>), dim3(grid), dim3(threads), lds, s, a, ca);
    } else {
      (void)hipFuncSetAttribute((const void *)k_embed_bwd_cells<W1, W2, W3, P, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_embed_bwd_cells<W1, W2, W3, P, false>), dim3(grid), dim3(threads), lds, s, a, ca);
    }
  }
}

bool embed_cells_config(const MixArgs &a, int want, int need, int *cap, int *threads, size_t *lds) {
  if (need < 1 || want < need || want > 255) return false;
  const int nnets = a.d.ntypes * a.d.ntypes;
  int id = 0;
#define X(a_, b_, c_, l_)                                                         \
  if (a.shape == id) return cells_config_t<a_, b_, c_, l_>(nnets, a.tab != nullptr, want, need, cap, threads, lds); \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
  return false;
}

int cells_grid(int64_t ncell) {
  int64_t g = ncell < 2048 ? ncell : 2048;
  return (int)(g < 1 ? 1 : g);
}

void launch_embed_cells(hipStream_t s, const MixArgs &a, const CellArgs &ca, int grid, int threads, size_t lds) {
  int id = 0;
#define X(a_, b_, c_, l_)                                                          \
  if (a.shape == id) {                                                             \
    if (a.prec == 0) launch_cells_t<a_, b_, c_, l_, 0>(s, a, ca, grid, threads, lds); \
    else launch_cells_t<a_, b_, c_, l_, 1>(s, a, ca, grid, threads, lds);          \
    return;                                                                        \
  }                                                                                \
  ++id;
  DPK_MIX_SHAPES(X)
#undef X
}

void launch_cell_gather(hipStream_t s, const CellArgs &ca, double *F) {
  if (ca.n <= 0) return;
  hipLaunchKernelGGL(k_cell_gather, dim3((unsigned)((ca.n + 255) / 256)), dim3(256), 0, s, ca, F);
}

}  // namespace dpk
