// Deterministic FP64 reductions (energy, virial, kinetic energy) and the
// velocity-Verlet integrator with thermo rows (Section VI: NVE MD loop,
// thermo output every 20 steps).  Units A, fs, amu, eV; a = F/m * conv with
// conv = 1/103.6427 (eV/A/amu -> A/fs^2).
#include "dp_internal.h"

namespace dpk {

constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;

__device__ inline double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  __syncthreads();
  return t;  // valid in thread 0
}

// stage 1: block b sums a fixed contiguous chunk; stage 2 sums the partials
__global__ void __launch_bounds__(RED_THREADS) k_sum_stage1(const double *x, int64_t n, double *partial) {
  __shared__ double sh[RED_THREADS / 64];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b = (int64_t)blockIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  double v = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += RED_THREADS) v += x[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

__global__ void __launch_bounds__(RED_THREADS) k_sum_stage2(const double *partial, int np, double *out, double scale) {
  __shared__ double sh[RED_THREADS / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += RED_THREADS) v += partial[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[0] = v * scale;
}

void launch_sum(hipStream_t s, const double *x, int64_t n, double *partial, double *out, double scale) {
  hipLaunchKernelGGL(k_sum_stage1, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, partial);
  hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(RED_THREADS), 0, s, partial, RED_BLOCKS, out, scale);
}

__global__ void __launch_bounds__(RED_THREADS) k_sum9(const double *part, int np, double *out) {
  __shared__ double sh[RED_THREADS / 64];
  for (int k = 0; k < 9; ++k) {
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += RED_THREADS) v += part[(int64_t)i * 9 + k];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[k] = v;
  }
}

void launch_sum9(hipStream_t s, const double *part, int nparts, double *out) {
  hipLaunchKernelGGL(k_sum9, dim3(1), dim3(RED_THREADS), 0, s, part, nparts, out);
}

__global__ void k_zero(double *x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

void launch_zero(hipStream_t s, double *x, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
}

struct TypeScale {
  double v[MAXT];
};

__global__ void k_verlet_half(int64_t n, double *v, const double *f, const int32_t *types, TypeScale c,
                              double half_dt, const uint32_t *flags, long long *fault_step, long long step) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (*flags & FLAG_HALT) {
    if (i == 0 && fault_step && *fault_step < 0) *fault_step = step;
    return;
  }
  if (i >= 3 * n) return;
  v[i] += half_dt * f[i] * c.v[types[i / 3]];
}

void launch_verlet_half(hipStream_t s, int64_t n, double *v, const double *f, const int32_t *types,
                        const double *inv_m_conv, double half_dt, const uint32_t *flags, long long *fault_step,
                        int64_t step) {
  TypeScale c{};
  for (int t = 0; t < MAXT; ++t) c.v[t] = inv_m_conv[t];
  if (n > 0)
    hipLaunchKernelGGL(k_verlet_half, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, n, v, f, types, c,
                       half_dt, flags, fault_step, (long long)step);
}

__global__ void k_verlet_drift(int64_t n, double *x, const double *v, double dt, double L0, double L1, double L2,
                               const uint32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n || (*flags & FLAG_HALT)) return;
  const int a = (int)(i % 3);
  const double L = a == 0 ? L0 : (a == 1 ? L1 : L2);
  double y = x[i] + dt * v[i];
  y = y - L * floor(y / L);
  if (y >= L) y = 0.0;
  x[i] = y;
}

void launch_verlet_drift(hipStream_t s, int64_t n, double *x, const double *v, double dt, const double *L,
                         const uint32_t *flags) {
  if (n > 0)
    hipLaunchKernelGGL(k_verlet_drift, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, n, x, v, dt, L[0],
                       L[1], L[2], flags);
}

__global__ void __launch_bounds__(RED_THREADS) k_kinetic1(int64_t n, const double *v, const int32_t *types,
                                                          TypeScale m, double *partial) {
  __shared__ double sh[RED_THREADS / 64];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b = (int64_t)blockIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  double acc = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += RED_THREADS) {
    const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
    acc += m.v[types[i]] * (vx * vx + vy * vy + vz * vz);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

void launch_kinetic(hipStream_t s, int64_t n, const double *v, const int32_t *types, const double *mass,
                    double *partial, double *out) {
  TypeScale m{};
  for (int t = 0; t < MAXT; ++t) m.v[t] = mass[t];
  hipLaunchKernelGGL(k_kinetic1, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, n, v, types, m, partial);
  // KE = 1/2 sum m v^2 * 103.6427 eV
  hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(RED_THREADS), 0, s, partial, RED_BLOCKS, out, 0.5 * 103.642696562);
}

__global__ void k_thermo_row(double *row, double step, const double *ke, const double *pe, const double *vir,
                             double ndof_kb, double inv3v, uint32_t *flags) {
  if (threadIdx.x != 0) return;
  const double k = ke[0], p = pe[0];
  row[0] = step;
  row[1] = k;
  row[2] = p;
  row[3] = k + p;
  row[4] = 2.0 * k / ndof_kb;
  row[5] = (2.0 * k + vir[0] + vir[4] + vir[8]) * inv3v;
  if (!isfinite(k + p)) atomicOr(flags, FLAG_NONFINITE);
}

void launch_thermo_row(hipStream_t s, double *row, double step, const double *ke, const double *pe, const double *vir,
                       double ndof_kb, double inv3v, uint32_t *flags) {
  hipLaunchKernelGGL(k_thermo_row, dim3(1), dim3(64), 0, s, row, step, ke, pe, vir, ndof_kb, inv3v, flags);
}

}  // namespace dpk
