// FP64 matrix-core layer helpers shared by the FP64 embedding kernels and
// the student's FP64 teacher (k_embed_f64.hip, k_student.hip).  Not part of
// the public ABI.
//
// Matrix layout: each layer is computed transposed, Z^T[out x 16] = W^T H^T,
// with 16 samples (neighbours of a tile) as the MFMA N dimension.  For
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

// Output tiles mt0 .. mt0 + EMB_G - 1 of one layer, acc[ct][g] = (W^T H^T)
// for column tile ct and output tile mt0 + g (a tile past the layer's last
// reads the last tile's weights; the caller discards it).  The B operand
// (activations, LDS) of a k-step feeds EMB_G tiles; every weight load is
// unconditional.  Weights stream from L2 in their padded [K][M] layout.
// KP > 0: the layer's shape is known at compile time, the k-loop is
// unrolled and each k-step's weights are loaded one k-step ahead.
template <int NCT, int KP, int MP>
__device__ inline void mfma_group_t(const double *__restrict__ W, int kp, int mp, const double *Hin, int cols,
                                    int lane, int mt0, v4d (&acc)[NCT][EMB_G]) {
  if constexpr (KP > 0) {
    kp = KP;
    mp = MP;
  }
  const int nmt = mp >> 4;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int g = 0; g < EMB_G; ++g) acc[ct][g] = v4d{0.0, 0.0, 0.0, 0.0};
  const double *wr = W + (size_t)(lane >> 4) * mp + (lane & 15);
  const double *hr = Hin + (lane >> 4) * cols + (lane & 15);
  int col[EMB_G];
#pragma unroll
  for (int g = 0; g < EMB_G; ++g) col[g] = 16 * (mt0 + g < nmt ? mt0 + g : nmt - 1);
  if constexpr (KP > 0) {
    double an[EMB_G];
#pragma unroll
    for (int g = 0; g < EMB_G; ++g) an[g] = wr[col[g]];
#pragma unroll
    for (int kk = 0; kk < KP; kk += 4) {
      double ac[EMB_G];
#pragma unroll
      for (int g = 0; g < EMB_G; ++g) ac[g] = an[g];
      if (kk + 4 < KP)
#pragma unroll
        for (int g = 0; g < EMB_G; ++g) an[g] = wr[(size_t)(kk + 4) * MP + col[g]];
      double bv[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) bv[ct] = hr[kk * cols + ct * 16];
#pragma unroll
      for (int g = 0; g < EMB_G; ++g)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct][g] = mfma64(ac[g], bv[ct], acc[ct][g]);
    }
  } else {
    for (int kk = 0; kk < kp; kk += 4) {
      double ac[EMB_G];
#pragma unroll
      for (int g = 0; g < EMB_G; ++g) ac[g] = wr[(size_t)kk * mp + col[g]];
      double bv[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) bv[ct] = hr[kk * cols + ct * 16];
#pragma unroll
      for (int g = 0; g < EMB_G; ++g)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct][g] = mfma64(ac[g], bv[ct], acc[ct][g]);
    }
  }
}

// The layer shapes of the 1-25-50-100 and 1-16-32-100 nets take the
// compile-time loop, others the generic one (the branch is wave-uniform).
template <int NCT>
__device__ inline void mfma_group(const double *__restrict__ W, int kp, int mp, const double *Hin, int cols, int lane,
                                  int mt0, v4d (&acc)[NCT][EMB_G]) {
  if (kp == 28 && mp == 64) mfma_group_t<NCT, 28, 64>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else if (kp == 52 && mp == 112) mfma_group_t<NCT, 52, 112>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else if (kp == 16 && mp == 32) mfma_group_t<NCT, 16, 32>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else if (kp == 32 && mp == 112) mfma_group_t<NCT, 32, 112>(W, kp, mp, Hin, cols, lane, mt0, acc);
  else mfma_group_t<NCT, 0, 0>(W, kp, mp, Hin, cols, lane, mt0, acc);
}

__device__ inline int skip_src(int f, int in, int out) {
  // feature of the previous layer added by the skip connection, or -1
  if (out == in) return f;
  if (out == 2 * in) return f >= in ? f - in : f;
  return -1;
}

}  // namespace dpk
