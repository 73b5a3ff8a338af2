// Matrix-core layer helpers of the FP64-structured embedding kernels (FP64
// and FP32) and the student's FP64 teacher (k_embed_f64.hip,
// k_student.hip).  Not part of the public ABI.
//
// Matrix layout: a layer is computed transposed, Z^T[out x 16] = W^T H^T,
// with 16 samples (neighbours of a tile) as the MFMA N dimension, or, with
// the operands of the same loads swapped (HA), as Z[16 x out] = H W.  For
// v_mfma_f64_16x16x4: A lane l holds A[l%16][l/16], B lane l holds
// B[l/16][l%16], and D register r of lane l is D[4r + l/16][l%16] (the f64
// variant interleaves rows by register, unlike the f32-output variants).
#pragma once
#include "dp_internal.h"

namespace dpk {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int EMB_G = 4;  // output tiles per MFMA group

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Matrix-core traits of the two real types the FP64-structured kernels run
// in: double (DP_FP64) and float (DP_MIX_FP32, v_mfma_f32_16x16x4_f32 with
// the same A and B lane layouts).  row(r, g): row inside the 16-row output
// tile of register r of a lane in group g = lane / 16.
typedef float f4v __attribute__((ext_vector_type(4)));
template <typename Real>
struct MF;
template <>
struct MF<double> {
  typedef v4d acc;
  typedef double4 vec4;
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int r, int g) { return 4 * r + g; }
  __device__ static double tanh_(double x) { return tanh64(x); }
  __device__ static vec4 zero4() { return make_double4(0.0, 0.0, 0.0, 0.0); }
};
template <>
struct MF<float> {
  typedef f4v acc;
  typedef float4 vec4;
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int r, int g) { return 4 * g + r; }
  __device__ static float tanh_(float x) { return tanhf(x); }
  __device__ static vec4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};

// Output tiles mt0 .. mt0 + EMB_G - 1 of one layer, acc[ct][g] = (W^T H^T)
// for column tile ct and output tile mt0 + g (a tile past the layer's last
// reads the last tile's weights; the caller discards it).  The B operand
// (activations, LDS) of a k-step feeds EMB_G tiles; every weight load is
// unconditional.  Weights stream from L2 in their padded [K][M] layout.
// KP > 0: the layer's shape is known at compile time, the k-loop is
// unrolled and each k-step's weights are loaded one k-step ahead.
// bop(kk, ct): the B operand of k-step kk and column tile ct for this lane
// (row kk + lane / 16 of the layer input, column lane % 16 of tile ct).
// HA: the same loads with the operands swapped -- bop gives the A operand
// H[n = lane % 16][kk + lane / 16] and the weights are B, so acc holds
// Z = H W (neighbours as rows) instead of its transpose.
template <int NCT, int KP, int MP, bool HA, typename Real, class BOp>
__device__ inline void mfma_group_tb(const Real *__restrict__ W, int kp, int mp, BOp bop, int lane, int mt0,
                                     typename MF<Real>::acc (&acc)[NCT][EMB_G]) {
  auto mma = [](Real w, Real h, typename MF<Real>::acc c) {
    if constexpr (HA) return MF<Real>::mma(h, w, c);
    else return MF<Real>::mma(w, h, c);
  };
  if constexpr (KP > 0) {
    kp = KP;
    mp = MP;
  }
  const int nmt = mp >> 4;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int g = 0; g < EMB_G; ++g) acc[ct][g] = typename MF<Real>::acc{0, 0, 0, 0};
  const Real *wr = W + (size_t)(lane >> 4) * mp + (lane & 15);
  int col[EMB_G];
#pragma unroll
  for (int g = 0; g < EMB_G; ++g) col[g] = 16 * (mt0 + g < nmt ? mt0 + g : nmt - 1);
  if constexpr (KP > 0) {
    Real an[EMB_G];
#pragma unroll
    for (int g = 0; g < EMB_G; ++g) an[g] = wr[col[g]];
#pragma unroll
    for (int kk = 0; kk < KP; kk += 4) {
      Real ac[EMB_G];
#pragma unroll
      for (int g = 0; g < EMB_G; ++g) ac[g] = an[g];
      if (kk + 4 < KP)
#pragma unroll
        for (int g = 0; g < EMB_G; ++g) an[g] = wr[(size_t)(kk + 4) * MP + col[g]];
      Real bv[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) bv[ct] = bop(kk, ct);
#pragma unroll
      for (int g = 0; g < EMB_G; ++g)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct][g] = mma(ac[g], bv[ct], acc[ct][g]);
    }
  } else {
    for (int kk = 0; kk < kp; kk += 4) {
      Real ac[EMB_G];
#pragma unroll
      for (int g = 0; g < EMB_G; ++g) ac[g] = wr[(size_t)kk * mp + col[g]];
      Real bv[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) bv[ct] = bop(kk, ct);
#pragma unroll
      for (int g = 0; g < EMB_G; ++g)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct][g] = mma(ac[g], bv[ct], acc[ct][g]);
    }
  }
}

// the same with the B operands from an LDS tile [row][cols] (column tile ct
// at column 16 ct)
template <int NCT, int KP, int MP, typename Real>
__device__ inline void mfma_group_t(const Real *__restrict__ W, int kp, int mp, const Real *Hin, int cols,
                                    int lane, int mt0, typename MF<Real>::acc (&acc)[NCT][EMB_G]) {
  const Real *hr = Hin + (lane >> 4) * cols + (lane & 15);
  mfma_group_tb<NCT, KP, MP, false, Real>(
      W, kp, mp, [&](int kk, int ct) { return hr[kk * cols + ct * 16]; }, lane, mt0, acc);
}

// The layer shapes of the 1-25-50-100 and 1-16-32-100 nets take the
// compile-time loop, others the generic one (the branch is wave-uniform).
template <int NCT, typename Real>
__device__ inline void mfma_group(const Real *__restrict__ W, int kp, int mp, const Real *Hin, int cols, int lane,
                                  int mt0, typename MF<Real>::acc (&acc)[NCT][EMB_G]) {
  if (kp == 28 && mp == 64) mfma_group_t<NCT, 28, 64, Real>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else if (kp == 52 && mp == 112) mfma_group_t<NCT, 52, 112, Real>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else if (kp == 16 && mp == 32) mfma_group_t<NCT, 16, 32, Real>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else if (kp == 32 && mp == 112) mfma_group_t<NCT, 32, 112, Real>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else mfma_group_t<NCT, 0, 0, Real>(W, kp, mp, Hin, cols, lane, mt0, acc);
}

// the same dispatch with a B-operand functor (see mfma_group_tb)
template <int NCT, bool HA = false, typename Real, class BOp>
__device__ inline void mfma_group_b(const Real *__restrict__ W, int kp, int mp, BOp bop, int lane, int mt0,
                                    typename MF<Real>::acc (&acc)[NCT][EMB_G]) {
  if (kp == 28 && mp == 64) mfma_group_tb<NCT, 28, 64, HA, Real>(W, kp, mp, bop, lane, mt0, acc);
  else if (kp == 52 && mp == 112) mfma_group_tb<NCT, 52, 112, HA, Real>(W, kp, mp, bop, lane, mt0, acc);
  else if (kp == 16 && mp == 32) mfma_group_tb<NCT, 16, 32, HA, Real>(W, kp, mp, bop, lane, mt0, acc);
  else if (kp == 32 && mp == 112) mfma_group_tb<NCT, 32, 112, HA, Real>(W, kp, mp, bop, lane, mt0, acc);
  else mfma_group_tb<NCT, 0, 0, HA, Real>(W, kp, mp, bop, lane, mt0, acc);
}

__device__ inline int skip_src(int f, int in, int out) {
  // feature of the previous layer added by the skip connection, or -1
  if (out == in) return f;
  if (out == 2 * in) return f >= in ? f - in : f;
  return -1;
}

}  // namespace dpk
