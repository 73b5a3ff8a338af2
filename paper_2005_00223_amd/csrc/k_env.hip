// Environment matrix (the paper's "Environment" operator, Section V-B and
// Table III): for every real slot of the formatted list,
//   d = r_j - r_i (minimum image), r = |d|,
//   R = (s, s dx/r, s dy/r, s dz/r),  s = sw(r)/r,
//   sw = 1 (r < rcs), u^3 (-6u^2 + 15u - 10) + 1 (rcs <= r < rc), 0 (r >= rc),
//   u = (r - rcs)/(rc - rcs)  (quintic switch, C2 in the displacements).
// Output rt[i][slot] = R and dr[i][slot] = (dx, dy, dz, r), double; for the
// mixed-precision path R is stored rounded to FP32 instead (its kernels read
// nothing else of it) and dr is not stored (its force pass recomputes the
// displacement from the positions).  Padded slots are not written (every consumer stops
// at the real count).
//
// One wave per centre atom; the lanes stride over the atom's real slots so
// that the two output streams are written contiguously.  HBM-bound:
// per real slot 4 B nlist + 32 B neighbour position (L2/MALL) in, 64 B out
// (16 B with the FP32 R and no dr).
#include "dp_internal.h"

namespace dpk {

constexpr int ENV_BATCH = 4;  // gathers in flight per lane


__device__ inline void put_rt(double4 *rt, int64_t k, double a, double b, double c, double e) {
  rt[k] = make_double4(a, b, c, e);
}
__device__ inline void put_rt(float4 *rt, int64_t k, double a, double b, double c, double e) {
  rt[k] = make_float4((float)a, (float)b, (float)c, (float)e);
}

template <typename RT>
__global__ void __launch_bounds__(256) k_env(int64_t n, const double4 *__restrict__ xw, Dims d, double L0, double L1,
                                             double L2, const int32_t *__restrict__ nlist,
                                             const int32_t *__restrict__ nreal, RT *__restrict__ rt,
                                             double4 *__restrict__ dr) {
  int lane = threadIdx.x & 63;
  int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double4 p = xw[i];
  const double rc = d.rcut, rcs = d.rcut_smth, inv_w = 1.0 / (d.rcut - d.rcut_smth);
  for (int u = 0; u < d.ntypes; ++u) {
    int cnt = nreal[i * d.ntypes + u];
    int64_t base = i * (int64_t)d.nnei + d.off[u];
    for (int q0 = 0; q0 < cnt; q0 += 64 * ENV_BATCH) {
      // issue the list loads, then the position gathers, of ENV_BATCH rounds
      int jb[ENV_BATCH];
      double4 pb[ENV_BATCH];
#pragma unroll
      for (int v = 0; v < ENV_BATCH; ++v) {
        const int q = q0 + 64 * v + lane;
        jb[v] = nlist[base + (q < cnt ? q : cnt - 1)];  // unconditional; masked below
      }
#pragma unroll
      for (int v = 0; v < ENV_BATCH; ++v) pb[v] = xw[jb[v]];
#pragma unroll
      for (int v = 0; v < ENV_BATCH; ++v)
        if (q0 + 64 * v + lane >= cnt) jb[v] = -1;
#pragma unroll
      for (int v = 0; v < ENV_BATCH; ++v) {
        const int q = q0 + 64 * v + lane;
        if (jb[v] < 0) continue;
        const double4 pj = pb[v];
        const double4 D = pair_disp(p, pj, L0, L1, L2);
        const double s = env_s(D.w, rcs, rc, inv_w);
        const double t = s * (1.0 / D.w);
        put_rt(rt, base + q, s, t * D.x, t * D.y, t * D.z);
        if (dr) dr[base + q] = D;
      }
    }
  }
}

void launch_env(hipStream_t s, int64_t n, const double4 *xw, const Dims &d, const double *L, const int32_t *nlist,
                const int32_t *nreal, double4 *rt, float4 *rt32, double4 *dr) {
  if (n <= 0) return;
  if (rt32)
    hipLaunchKernelGGL(k_env<float4>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, xw, d, L[0], L[1], L[2],
                       nlist, nreal, rt32, dr);
  else
    hipLaunchKernelGGL(k_env<double4>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, xw, d, L[0], L[1], L[2],
                       nlist, nreal, rt, dr);
}

}  // namespace dpk
