// Wide embedding nets in mixed precision (the embedding-size study of the
// paper's Sec. VII-D / Fig. 7: last-layer matrices up to 1024 x 2048).
//
// Widths of 256 and more do not fit the register-resident per-neighbour
// kernels, so this path runs the embedding net over all real neighbour pairs
// as 16-bit MFMA GEMMs (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulation),
// the regime in which the paper found MIX-16 to scale with the matrix size:
//
//   count   pairs per (centre type, neighbour type) net, per-atom offsets
//   layer 0 1 -> W1 on the VALU: h = tanh(s w + b) and dh/ds = (1 - h^2) w
//   GEMMs   layer l >= 1: Z = H W_l over rows (value, tangent) interleaved,
//           epilogue h' = skip(h) + tanh(z + b), dh'/ds = skip(dh/ds) +
//           (1 - tanh^2) dz/ds  (forward-mode tangent, so dG/ds is carried
//           through the same GEMMs as G: no backward GEMMs are needed)
//   T       T_i = (1/Nc) sum_j G_j R_j^T per atom (FP32 sums)
//   (fitting net: the mixed fitting kernels, D = T T<^T formed on the fly)
//   bwd     per pair dE/dR_j = G_j^T dT_i, dE/ds_j = (dT_i R_j) . dG_j/ds,
//           then the FP64 force Jacobian, F_j atomics and the virial.
//
// Activations are stored in one of two ways.  By default each value is kept
// as a hi + lo pair of 16-bit numbers whose sum is the FP32 activation to
// about 2^-22 relative; every GEMM multiplies both halves by the same 16-bit
// weights (K runs over [hi | lo]) and T and the backward contract the two
// halves in turn (they are linear in G).  Forces then come within about
// 1e-5 relative of FP64 arithmetic on the same rounded weights.  The other
// storage (split = 0) keeps one 16-bit value per activation, the paper's
// MIX-16 scheme (Sec. V-B): half the products and activation bytes, with
// each pair's dE/dR within about two 16-bit roundings (2u) of the exact
// value.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "dp_wide.h"

namespace dpk {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int P> struct WT;
template <> struct WT<0> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  __device__ static v4f mma(v8 a, v8 b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
  __device__ static float get(uint16_t u) { return (float)__builtin_bit_cast(_Float16, u); }
  __device__ static uint16_t put(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
};
template <> struct WT<1> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  __device__ static v4f mma(v8 a, v8 b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __device__ static float get(uint16_t u) { return __builtin_bit_cast(float, (uint32_t)u << 16); }
  __device__ static uint16_t put(float x) {  // round to nearest even
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  }
};

template <int P>
__device__ inline uint4 pack8(const float (&x)[8]) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (uint32_t)WT<P>::put(x[2 * k]) | ((uint32_t)WT<P>::put(x[2 * k + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// 8 values as 16-bit hi = rn16(x) and lo = rn16(x - hi)
template <int P>
__device__ inline void pack8_split(const float (&x)[8], uint4 &hi, uint4 &lo) {
  float r[8];
  uint16_t h[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    h[q] = WT<P>::put(x[q]);
    r[q] = x[q] - WT<P>::get(h[q]);
  }
  hi = make_uint4((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                  (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16));
  lo = pack8<P>(r);
}

// the value of feature f of an activation row (split: hi + lo)
template <int P>
__device__ inline float act(const uint16_t *row, int f, int width, int split) {
  const float v = WT<P>::get(row[f]);
  return split ? v + WT<P>::get(row[width + f]) : v;
}

// ---------------------------------------------------------------------------
// pair counts: atom i's pairs of net (t_i, u) start at pair poff[i][u] of
// that net (wave prefix sums, one atomic per wave and net)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wide_count(WideArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, T = a.d.ntypes;
  const int t = i < a.n ? (int)a.xw[i].w : -1;
  for (int net = 0; net < T * T; ++net) {
    const int u = net % T;
    const bool mine = i < a.n && t == net / T;
    const int c = mine ? a.nreal[i * T + u] : 0;
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    const int total = __shfl(x, 63);
    int base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(a.cnt + net, total);
    base = __shfl(base, 63);
    if (mine) a.poff[i * T + u] = base + x - c;
  }
}

void launch_wide_count(hipStream_t s, const WideArgs &a) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_wide_count, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// layer 0 (1 -> W1): value and tangent rows of every real pair, 8 features
// per thread
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_wide_l0(WideArgs a) {
  const int T = a.d.ntypes, W1 = a.d.ew[1], C = W1 / 8;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int t = (int)a.xw[i].w;
    for (int u = 0; u < T; ++u) {
      const int net = t * T + u, nr = a.nreal[i * T + u];
      const int64_t rb = a.row0[net] + 2 * (int64_t)a.poff[i * T + u];
      const float4 *R = a.rt + i * a.d.nnei + a.d.off[u];
      const float *w0 = a.w0[net], *b0 = a.b0[net];
      for (int e = threadIdx.x; e < nr * C; e += blockDim.x) {
        const int k = e / C, c = e % C;
        const float s = R[k].x;
        float y[8], dy[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float w = w0[8 * c + q];
          const float h = tanh_f(s * w + b0[8 * c + q]);
          y[q] = h;
          dy[q] = (1.f - h * h) * w;
        }
        const int ld = W1 << a.split;  // row length
        uint16_t *row = a.X0 + (rb + 2 * k) * ld + 8 * c;
        if (a.split) {
          uint4 hi, lo;
          pack8_split<P>(y, hi, lo);
          *(uint4 *)row = hi;
          *(uint4 *)(row + W1) = lo;
          pack8_split<P>(dy, hi, lo);
          *(uint4 *)(row + ld) = hi;
          *(uint4 *)(row + ld + W1) = lo;
        } else {
          *(uint4 *)row = pack8<P>(y);
          *(uint4 *)(row + ld) = pack8<P>(dy);
        }
      }
    }
  }
}

void launch_wide_l0(hipStream_t s, const WideArgs &a) {
  if (a.n <= 0) return;
  const unsigned grid = (unsigned)(a.n < WIDE_GRID ? a.n : WIDE_GRID);
  if (a.prec == 0) hipLaunchKernelGGL(k_wide_l0<0>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_wide_l0<1>, dim3(grid), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// GEMM with the layer epilogue.  128 x 128 output tile per workgroup of four
// waves (2 x 2, 64 x 64 each = 4 x 4 MFMA tiles), K staged through LDS 64 at
// a time, double buffered.  The operands go global -> LDS by direct loads
// (global_load_lds_dwordx4, no registers): a 1 KB block holds 8 rows x 64 k,
// lane l loading 16 bytes of row l / 8 (eight lanes cover a row's 128
// contiguous bytes) into slot l; the 16-byte chunk c of row r sits in slot
// c ^ r of that row, so the eight rows a fragment read touches at one chunk
// fall on different banks.  Output lane (g, c) of an MFMA tile holds rows 4g..4g+3 of
// feature c: rows (4g, 4g+1) and (4g+2, 4g+3) are (value, tangent) pairs, so
// tanh and its derivative are applied there; the results are then staged in
// LDS (FP32) and written, with the skip connection added, 16 bytes per lane.
// ---------------------------------------------------------------------------
// tile shapes: BIG = 0: 128 x 128, four waves of 64 x 64; BIG = 1:
// 256 x 256, eight waves of 64 x 128 (more MFMA work per LDS byte read).
// Two stages: measured on the largest layer (K 1024, N 2048), three stages
// of 256 x 128 tiles ran 20% slower than two of 256 x 256.
template <int BIG>
struct GT {
  static constexpr int BM = BIG ? 256 : 128, BN = BIG ? 256 : 128, NT = BIG ? 8 : 4;  // NT: 16-col tiles per wave
  static constexpr int WM = BM / 64, WAVES = WM * (BN / (16 * NT));
  static constexpr int NSTAGE = 2;
  static constexpr int STAGE = 2 * (BM + BN) * WIDE_BK;  // bytes of one stage (A then B)
  static constexpr int NBLK = (BM + BN) / 8;             // 1 KB blocks per stage
  static constexpr int NBPW = NBLK / WAVES;              // blocks each wave loads per stage
  static_assert(NBLK == NBPW * WAVES, "equal shares of a stage");
  static_assert(NSTAGE * STAGE <= 160 * 1024, "stages fit the LDS");
};

// s_waitcnt with vmcnt(n) only (expcnt and lgkmcnt left at their maxima)
template <int n>
__device__ inline void wait_vmcnt() {
  __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

__device__ inline void wide_dma(const uint16_t *src, unsigned char *lds) {
  __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

template <int P, int BIG>
__global__ void __launch_bounds__(64 * GT<BIG>::WAVES, BIG ? 1 : 2) k_wide_gemm(WideGemm g, int nbm, int nbn) {
  typedef typename WT<P>::v8 V;
  typedef GT<BIG> S;
  constexpr int NT = S::NT;
  constexpr int NS = S::NSTAGE, NB = S::NBPW;
  __shared__ __align__(16) unsigned char lds[NS * S::STAGE];
  // workgroups are dealt round-robin to the eight XCDs: give each XCD a
  // contiguous run of tiles, ordered in groups of GM row blocks x all column
  // blocks, column block outer, so that an XCD's L2 holds the group's row
  // blocks (1024 rows x K) while the weight columns stream past once per group
  const int ntile = nbm * nbn, per = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= ntile) return;  // whole workgroup: before any barrier
  constexpr int GM = BIG ? 4 : 8;
  const int grp = tile / (GM * nbn), in = tile % (GM * nbn);
  const int gm = nbm - grp * GM < GM ? nbm - grp * GM : GM;
  const int bm = grp * GM + in % gm, bn = in / gm;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv % S::WM, wn = wv / S::WM;
  const int K = g.K, Kb = g.Kb, N = g.N, ldy = g.N << g.split;
  // blocks of a stage: A rows 8 b..8 b+7 in block b (b < BM / 8), then the B
  // rows; wave w loads blocks w + WAVES j, lane l row l / 8, chunk (l % 8) ^ (l / 8)
  const int fr = lane & 15;
  const uint16_t *src[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int b = wv + S::WAVES * j, isb = b >= S::BM / 8, rb = isb ? b - S::BM / 8 : b;
    const uint16_t *base = isb ? g.Bt + (int64_t)bn * S::BN * Kb : g.A + (int64_t)bm * S::BM * K;
    src[j] = base + (int64_t)(8 * rb + (lane >> 3)) * (isb ? Kb : K) + 8 * ((lane & 7) ^ (lane >> 3));
  }
  // the B rows hold Kb values: a split input's second half reuses them
  bool bblk[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) bblk[j] = wv + S::WAVES * j >= S::BM / 8;
  // fragment reads: row fr of a 16-row group = block 2 group + fr / 8, row fr % 8,
  // chunk 4 ks + lane / 16 at slot chunk ^ (fr % 8)
  const int rr = fr & 7, rbk = fr >> 3;
  auto issue = [&](int kt, int st) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      wide_dma(src[j] + (bblk[j] ? (kt * WIDE_BK) % Kb : kt * WIDE_BK), lds + st * S::STAGE + (wv + S::WAVES * j) * 1024);
  };
  v4f acc[4][NT];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) acc[mi][ni] = v4f{0.f, 0.f, 0.f, 0.f};
  const int nkt = K / WIDE_BK;
  issue(0, 0);
  if (NS > 2 && nkt > 1) issue(1, 1);
  for (int kt = 0; kt < nkt; ++kt) {
    // stage kt has landed for this wave (with three stages the next one may
    // still be in flight), then for all waves; the buffer refilled below was
    // last read in iteration kt - 1, which every wave has finished
    if (NS > 2 && kt + 1 < nkt) wait_vmcnt<NB>();
    else wait_vmcnt<0>();
    __syncthreads();
    if (kt + NS - 1 < nkt) issue(kt + NS - 1, (kt + NS - 1) % NS);
    const unsigned char *sb = lds + (kt % NS) * S::STAGE;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int off = (rr * 8 + ((4 * ks + (lane >> 4)) ^ rr)) * 16 + rbk * 1024;
      V af[4], bf[NT];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) af[mi] = *(const V *)(sb + 2 * (4 * wm + mi) * 1024 + off);
#pragma unroll
      for (int ni = 0; ni < NT; ++ni) bf[ni] = *(const V *)(sb + (S::BM / 8 + 2 * (NT * wn + ni)) * 1024 + off);
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < NT; ++ni) acc[mi][ni] = WT<P>::mma(af[mi], bf[ni], acc[mi][ni]);
    }
  }
  __syncthreads();  // the stages are no longer read: the epilogue reuses the LDS
  // epilogue, 16 rows at a time: y = tanh(z + b) and dy = (1 - tanh^2) dz in
  // the MFMA layout -> LDS (16 rows x the wave's 16 NT columns, FP32) -> per
  // lane 8 consecutive columns of one row, plus the skip, out; a store
  // instruction covers whole rows of the wave's columns (full 128-byte lines)
  constexpr int EPS = 16 * NT + 4;  // FP32 row stride of the staging (bank spread)
  constexpr int CPR = 2 * NT;       // lanes per row (8 columns each)
  constexpr int RPI = 64 / CPR;     // rows per store instruction
  float *ep = (float *)lds + wv * 16 * EPS;
  const int g4 = lane >> 4, cq = lane % CPR, rq = lane / CPR;
  const int64_t row0 = (int64_t)bm * S::BM + 64 * wm;
  const int n = bn * S::BN + 16 * NT * wn + 8 * cq;
  const int sc = g.skip == 1 ? n : (n < Kb ? n : n - Kb);
  float bias[NT];
#pragma unroll
  for (int ni = 0; ni < NT; ++ni) bias[ni] = g.bias[bn * S::BN + 16 * NT * wn + 16 * ni + fr];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi) {
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) {
      const v4f c = acc[mi][ni];
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const float h = tanh_f(c[2 * pr] + bias[ni]);
        const int r = 4 * g4 + 2 * pr;
        ep[r * EPS + 16 * ni + fr] = h;
        ep[(r + 1) * EPS + 16 * ni + fr] = (1.f - h * h) * c[2 * pr + 1];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int it = 0; it < 16 / RPI; ++it) {
      const int r = RPI * it + rq;
      const float4 y0 = *(const float4 *)(ep + r * EPS + 8 * cq);
      const float4 y1 = *(const float4 *)(ep + r * EPS + 8 * cq + 4);
      float y[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
      const int64_t row = row0 + 16 * mi + r;
      if (g.skip) {
#pragma unroll
        for (int half = 0; half <= g.split; ++half) {
          const uint4 hv = *(const uint4 *)(g.A + row * K + half * Kb + sc);
          const uint32_t hw[4] = {hv.x, hv.y, hv.z, hv.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) y[q] += WT<P>::get((uint16_t)(hw[q >> 1] >> (16 * (q & 1))));
        }
      }
      if (g.split) {
        uint4 hi, lo;
        pack8_split<P>(y, hi, lo);
        *(uint4 *)(g.Y + row * ldy + n) = hi;
        *(uint4 *)(g.Y + row * ldy + N + n) = lo;
      } else {
        *(uint4 *)(g.Y + row * ldy + n) = pack8<P>(y);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

void launch_wide_gemm(hipStream_t s, const WideGemm &g, int prec) {
  if (g.rows <= 0) return;
  if (g.N % GT<1>::BN == 0 && g.rows % GT<1>::BM == 0) {
    typedef GT<1> S;
    const int nbm = (int)(g.rows / S::BM), nbn = g.N / S::BN;
    const unsigned grid = (unsigned)((nbm * nbn + 7) / 8 * 8);
    if (prec == 0) hipLaunchKernelGGL((k_wide_gemm<0, 1>), dim3(grid), dim3(64 * S::WAVES), 0, s, g, nbm, nbn);
    else hipLaunchKernelGGL((k_wide_gemm<1, 1>), dim3(grid), dim3(64 * S::WAVES), 0, s, g, nbm, nbn);
    return;
  }
  typedef GT<0> S;
  const int nbm = (int)(g.rows / S::BM), nbn = g.N / S::BN;
  const unsigned grid = (unsigned)((nbm * nbn + 7) / 8 * 8);
  if (prec == 0) hipLaunchKernelGGL((k_wide_gemm<0, 0>), dim3(grid), dim3(64 * S::WAVES), 0, s, g, nbm, nbn);
  else hipLaunchKernelGGL((k_wide_gemm<1, 0>), dim3(grid), dim3(64 * S::WAVES), 0, s, g, nbm, nbn);
}

// ---------------------------------------------------------------------------
// T_i = (1/Nc) sum_j G_j R_j^T.  Thread (group, c) sums features 8c..8c+7
// over the pairs k = group (mod groups); the groups' partial sums are added
// in group order.
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_wide_T(WideArgs a) {
  __shared__ float4 part[256 * 8];
  const int T = a.d.ntypes, M1 = a.d.M1, C = M1 / 8, NG = 256 / C;
  const int tid = threadIdx.x, c = tid % C, grp = tid / C;
  // when C does not divide 256 the threads past NG * C have no group: they
  // neither sum nor store (they still reach every barrier)
  const bool active = grp < NG;
  const float inv_nc = (float)a.d.inv_nc;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const int t = (int)a.xw[i].w;
    float4 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int u = 0; u < T && active; ++u) {
      const int net = t * T + u, nr = a.nreal[i * T + u];
      const int64_t rb = a.row0[net] + 2 * (int64_t)a.poff[i * T + u];
      const float4 *R = a.rt + i * a.d.nnei + a.d.off[u];
      const int ld = M1 << a.split;  // row length; T is linear in G: hi and lo rows add
#pragma unroll 4
      for (int e = grp; e < (nr << a.split); e += NG) {
        const int k = e >> a.split, half = e & a.split;
        const uint4 gv = *(const uint4 *)(a.G + (rb + 2 * k) * ld + half * M1 + 8 * c);
        const float4 r = R[k];
        const uint32_t w[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float x = WT<P>::get((uint16_t)(w[q >> 1] >> (16 * (q & 1))));
          acc[q].x += x * r.x;
          acc[q].y += x * r.y;
          acc[q].z += x * r.z;
          acc[q].w += x * r.w;
        }
      }
    }
    float4 *Tg = (float4 *)(a.T32 + (i * M1 + 8 * c) * 4);
    if (NG == 1) {
      if (!active) continue;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        Tg[q] = make_float4(acc[q].x * inv_nc, acc[q].y * inv_nc, acc[q].z * inv_nc, acc[q].w * inv_nc);
      continue;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) part[tid * 8 + q] = acc[q];
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float4 v = part[c * 8 + q];
        for (int h = 1; h < NG; ++h) {
          const float4 p = part[(h * C + c) * 8 + q];
          v.x += p.x;
          v.y += p.y;
          v.z += p.z;
          v.w += p.w;
        }
        Tg[q] = make_float4(v.x * inv_nc, v.y * inv_nc, v.z * inv_nc, v.w * inv_nc);
      }
    }
    __syncthreads();
  }
}

void launch_wide_T(hipStream_t s, const WideArgs &a) {
  if (a.n <= 0) return;
  const unsigned grid = (unsigned)(a.n < WIDE_GRID ? a.n : WIDE_GRID);
  if (a.prec == 0) hipLaunchKernelGGL(k_wide_T<0>, dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_wide_T<1>, dim3(grid), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// backward: per pair gR = G^T dT (4 values) and gs = (dT R) . dG/ds, summed
// over features by the wave (lane l takes features 4l + 256m); every 64
// pairs each lane runs the FP64 force pass of one of them.  dT of the atom
// is staged in LDS.
// ---------------------------------------------------------------------------
template <int P, int NS, int SP>
__global__ void __launch_bounds__(256) k_wide_bwd(WideArgs a) {
  __shared__ float4 dts[2048];
  __shared__ double vred[4][9];
  const int T = a.d.ntypes, M1 = 256 * NS;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double rc = a.d.rcut, rcs = a.d.rcut_smth, inv_w = 1.0 / (rc - rcs);
  double vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    __syncthreads();  // the previous atom's dT is no longer read
    const float4 *dTg = (const float4 *)(a.dT32 + i * M1 * 4);
    for (int f = tid; f < M1; f += 256) dts[f] = dTg[f];
    __syncthreads();
    const int t = (int)a.xw[i].w;
    int nru[WIDE_MAXT], np = 0;
    for (int u = 0; u < T; ++u) {
      nru[u] = a.nreal[i * T + u];
      np += nru[u];
    }
    if (wv * 64 >= np) continue;
    const double4 xi = a.xw[i];
    double fi0 = 0.0, fi1 = 0.0, fi2 = 0.0;
    for (int q0 = wv * 64; q0 < np; q0 += 256) {
      const int nq = np - q0 < 64 ? np - q0 : 64;
      float4 mine = make_float4(0.f, 0.f, 0.f, 0.f);
      int64_t mslot = 0;
      for (int jj = 0; jj < nq; ++jj) {
        int u = 0, k = q0 + jj;
        while (k >= nru[u]) k -= nru[u++];
        const int net = t * T + u;
        const int64_t row = a.row0[net] + 2 * ((int64_t)a.poff[i * T + u] + k);
        const int64_t slot = i * a.d.nnei + a.d.off[u] + k;
        const float4 R = a.rt[slot];
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, gs = 0.f;
        // gR and gs are linear in G and dG/ds: with split rows the hi and lo
        // halves are contracted one after the other
        constexpr int ld = M1 << SP;
#pragma unroll 1
        for (int half = 0; half <= SP; ++half) {
          const uint16_t *gv0 = a.G + row * ld + half * M1, *gt0 = gv0 + ld;
          // steps whose loads are in flight together: all of them up to 4, else
          // the largest divisor of NS up to 4 (register budget)
          constexpr int MG = NS <= 4 ? NS : (NS % 4 == 0 ? 4 : (NS % 3 == 0 ? 3 : (NS % 2 == 0 ? 2 : 1)));
#pragma unroll 1
          for (int m0 = 0; m0 < NS; m0 += MG) {
            uint2 hv[MG], ht[MG];
#pragma unroll
            for (int m = 0; m < MG; ++m) {
              hv[m] = *(const uint2 *)(gv0 + 4 * lane + 256 * (m0 + m));
              ht[m] = *(const uint2 *)(gt0 + 4 * lane + 256 * (m0 + m));
            }
#pragma unroll
            for (int m = 0; m < MG; ++m) {
              const int f = 4 * lane + 256 * (m0 + m);
              const uint32_t wv4[2] = {hv[m].x, hv[m].y}, wt4[2] = {ht[m].x, ht[m].y};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const float x = WT<P>::get((uint16_t)(wv4[e >> 1] >> (16 * (e & 1))));
                const float xt = WT<P>::get((uint16_t)(wt4[e >> 1] >> (16 * (e & 1))));
                const float4 d = dts[f + e];
                g0 += x * d.x;
                g1 += x * d.y;
                g2 += x * d.z;
                g3 += x * d.w;
                gs += xt * (d.x * R.x + d.y * R.y + d.z * R.z + d.w * R.w);
              }
            }
          }
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          g0 += __shfl_xor(g0, o);
          g1 += __shfl_xor(g1, o);
          g2 += __shfl_xor(g2, o);
          g3 += __shfl_xor(g3, o);
          gs += __shfl_xor(gs, o);
        }
        if (lane == jj) {
          mine = make_float4(g0 + gs, g1, g2, g3);
          mslot = slot;
        }
      }
      if (lane < nq) {
        const int j = a.nlist[mslot];
        if (a.net_deriv) {
          double *nd = a.net_deriv + mslot * 4;
          nd[0] = mine.x;
          nd[1] = mine.y;
          nd[2] = mine.z;
          nd[3] = mine.w;
        }
        double gx, gy, gz;
        pair_force(pair_disp_sq(xi, a.xw[j], a.L[0], a.L[1], a.L[2]), mine, rc, rcs, inv_w, gx, gy, gz, fi0, fi1, fi2,
                   vir);
        unsafeAtomicAdd(a.force + 3 * (int64_t)j + 0, -gx);
        unsafeAtomicAdd(a.force + 3 * (int64_t)j + 1, -gy);
        unsafeAtomicAdd(a.force + 3 * (int64_t)j + 2, -gz);
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      fi0 += __shfl_xor(fi0, o);
      fi1 += __shfl_xor(fi1, o);
      fi2 += __shfl_xor(fi2, o);
    }
    if (lane == 0) {
      unsafeAtomicAdd(a.force + 3 * i + 0, fi0);
      unsafeAtomicAdd(a.force + 3 * i + 1, fi1);
      unsafeAtomicAdd(a.force + 3 * i + 2, fi2);
    }
  }
  // block partial of the virial (lanes, then waves in order)
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double v = vir[k];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    if (lane == 0) vred[wv][k] = v;
  }
  __syncthreads();
  if (tid < 9) a.vir_part[(int64_t)blockIdx.x * 9 + tid] = ((vred[0][tid] + vred[1][tid]) + vred[2][tid]) + vred[3][tid];
}

void launch_wide_bwd(hipStream_t s, const WideArgs &a) {
  if (a.n <= 0) return;
  const unsigned grid = (unsigned)(a.n < WIDE_GRID ? a.n : WIDE_GRID);
  // M1 = 256 NS, NS = 1..8 (the widths the path takes)
  switch (a.d.M1 / 256) {
#define WIDE_BWD_CASE(ns)                                                                                  \
  case ns:                                                                                                 \
    if (a.split) {                                                                                         \
      if (a.prec == 0) hipLaunchKernelGGL((k_wide_bwd<0, ns, 1>), dim3(grid), dim3(256), 0, s, a);        \
      else hipLaunchKernelGGL((k_wide_bwd<1, ns, 1>), dim3(grid), dim3(256), 0, s, a);                    \
    } else {                                                                                               \
      if (a.prec == 0) hipLaunchKernelGGL((k_wide_bwd<0, ns, 0>), dim3(grid), dim3(256), 0, s, a);        \
      else hipLaunchKernelGGL((k_wide_bwd<1, ns, 0>), dim3(grid), dim3(256), 0, s, a);                    \
    }                                                                                                      \
    break;
    WIDE_BWD_CASE(1) WIDE_BWD_CASE(2) WIDE_BWD_CASE(3) WIDE_BWD_CASE(4) WIDE_BWD_CASE(5) WIDE_BWD_CASE(6)
    WIDE_BWD_CASE(7) WIDE_BWD_CASE(8)
#undef WIDE_BWD_CASE
    default: break;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
bool wide_supported(const Dims &d, const char **why) {
  if (d.ntypes > WIDE_MAXT) return *why = "wide embedding nets take at most 4 atom types", false;
  if (d.n_emb < 2) return *why = "wide embedding nets need two or more layers", false;
  if (d.emb_lin) return *why = "wide embedding nets need a tanh last layer", false;
  for (int l = 1; l < d.n_emb; ++l) {
    if (d.ew[l] % WIDE_BK != 0) return *why = "wide embedding: hidden widths must be multiples of 64", false;
    if (d.ew[l + 1] % WIDE_BN != 0) return *why = "wide embedding: widths after layer 1 must be multiples of 128", false;
  }
  if (d.M1 % 256 != 0 || d.M1 > 2048) return *why = "wide embedding: M1 must be a multiple of 256, at most 2048", false;
  return true;
}

static uint16_t bits16(double v, int prec) {
  const float f = (float)v;
  if (prec == 0) {
    const _Float16 h = (_Float16)f;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
  }
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

void wide_pack_net(const Dims &d, const double *const *W, const double *const *b, int prec,
                   std::vector<unsigned char> &buf, WideNet &o) {
  auto grow = [&](size_t bytes) {
    const size_t at = (buf.size() + 255) / 256 * 256;
    buf.resize(at + bytes, 0);
    return (int64_t)at;
  };
  for (int l = 0; l < d.n_emb; ++l) {
    const int in = d.ew[l], out = d.ew[l + 1];
    if (l == 0) {
      o.w[0] = grow(sizeof(float) * out);
      for (int f = 0; f < out; ++f) {
        const float v = (float)W[0][f];
        std::memcpy(buf.data() + o.w[0] + 4 * f, &v, 4);
      }
    } else {
      o.w[l] = grow(sizeof(uint16_t) * (size_t)in * out);
      for (int n = 0; n < out; ++n)
        for (int k = 0; k < in; ++k) {
          const uint16_t v = bits16(W[l][(size_t)k * out + n], prec);
          std::memcpy(buf.data() + o.w[l] + 2 * ((size_t)n * in + k), &v, 2);
        }
    }
    o.b[l] = grow(sizeof(float) * out);
    for (int f = 0; f < out; ++f) {
      const float v = (float)b[l][f];
      std::memcpy(buf.data() + o.b[l] + 4 * f, &v, 4);
    }
  }
}

}  // namespace dpk
