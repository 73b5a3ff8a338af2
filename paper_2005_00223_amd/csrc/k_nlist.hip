// Neighbour-list kernels: periodic wrap, per-type row ordering, cell list,
// skin candidate list and the formatted list of Section V-B (type-sorted,
// distance-sorted with index tie-break, nearest sel per type kept, -1
// padded).  The distance of every pair is the IEEE result of
//   d = x_j - x_i (one minimum-image correction), r = sqrt((dx dx + dy dy) + dz dz)
// in exactly this order; this file is compiled with -ffp-contract=off so no
// multiply-add is fused and the list is reproducible bit for bit.
//
// The paper packs (type, floor(|r| 1e8), j) into one 64-bit decimal key
// before sorting.  Here the same lexicographic order is bit-packed:
// type in bits 58..63, floor(r 1e8) in bits 26..57, j in bits 0..25, which
// bounds rc < 42.9 A and n < 2^26 (checked by the host).
#include <cmath>

#include "dp_internal.h"

namespace dpk {

__device__ inline double wrap1(double x, double L) {
  double y = x - L * floor(x / L);
  if (y >= L) y = 0.0;
  return y;
}

__device__ inline double min_image(double v, double L) {
  // selects, not branches: the same values without a divergent branch per
  // axis and candidate
  const double h = 0.5 * L, up = v - L, dn = v + L;
  return v > h ? up : (v < -h ? dn : v);
}

__global__ void k_wrap(int64_t n, const double *__restrict__ x, const int32_t *__restrict__ types, int ntypes,
                       double L0, double L1, double L2, double4 *__restrict__ xw, uint32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int t = types[i];
  if (t < 0 || t >= ntypes) {
    atomicOr(flags, FLAG_BAD_TYPE);
    t = 0;
  }
  double4 o;
  o.x = wrap1(x[3 * i + 0], L0);
  o.y = wrap1(x[3 * i + 1], L1);
  o.z = wrap1(x[3 * i + 2], L2);
  o.w = (double)t;
  xw[i] = o;
}

void launch_wrap(hipStream_t s, int64_t n, const double *coords, const int32_t *types, int ntypes, const double *L,
                 double4 *xw, uint32_t *flags) {
  if (n <= 0) return;
  int bs = 256;
  hipLaunchKernelGGL(k_wrap, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, n, coords, types, ntypes, L[0],
                     L[1], L[2], xw, flags);
}

// ---------------------------------------------------------------------------
// per-type row order: atoms of type t occupy rows type_start[t] + rank, with
// rank the index order inside the type and each type's block padded to
// ROW_TILE rows (padding rows have atom_of_pos = -1).
// ---------------------------------------------------------------------------
constexpr int TS_BLOCK = 256;

// mask (may be NULL): only atoms with mask[i] != 0 get rows
__global__ void k_type_count(int64_t n, const double4 *__restrict__ xw, int ntypes, int32_t *blk_counts,
                             const int32_t *mask) {
  __shared__ int32_t c[MAXT];
  if (threadIdx.x < MAXT) c[threadIdx.x] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * TS_BLOCK + threadIdx.x;
  if (i < n && (!mask || mask[i])) atomicAdd(&c[(int)xw[i].w], 1);
  __syncthreads();
  if (threadIdx.x < ntypes) blk_counts[(int64_t)blockIdx.x * MAXT + threadIdx.x] = c[threadIdx.x];
}

// single block: exclusive scan of block counts per type, padded type starts
__global__ void k_type_scan(int nblk, int ntypes, int32_t *blk_counts, int32_t *type_count, int32_t *type_start) {
  __shared__ int32_t tot[MAXT];
  int t = threadIdx.x;
  if (t < ntypes) {
    int32_t run = 0;
    for (int b = 0; b < nblk; ++b) {
      int32_t v = blk_counts[(int64_t)b * MAXT + t];
      blk_counts[(int64_t)b * MAXT + t] = run;
      run += v;
    }
    tot[t] = run;
    type_count[t] = run;
  }
  __syncthreads();
  if (t == 0) {
    int32_t s = 0;
    for (int u = 0; u < ntypes; ++u) {
      type_start[u] = s;
      s += (tot[u] + ROW_TILE - 1) / ROW_TILE * ROW_TILE;
    }
    type_start[ntypes] = s;
  }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_type_place(int64_t n, const double4 *__restrict__ xw, int ntypes, const int32_t *blk_off,
                             const int32_t *type_start, int32_t *pos_of_atom, int32_t *atom_of_pos,
                             const int32_t *mask) {
  __shared__ int32_t wtot[TS_BLOCK / 64][MAXT];
  int64_t i = (int64_t)blockIdx.x * TS_BLOCK + threadIdx.x;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int t = (i < n && (!mask || mask[i])) ? (int)xw[i].w : -1;
  int myrank = 0;
  for (int u = 0; u < ntypes; ++u) {
    unsigned long long m = __ballot(t == u);
    if (lane == 0) wtot[wv][u] = __popcll(m);
    if (t == u) myrank = __popcll(m & ((1ull << lane) - 1ull));
  }
  __syncthreads();
  if (t >= 0) {
    for (int w = 0; w < wv; ++w) myrank += wtot[w][t];
    int32_t pos = type_start[t] + blk_off[(int64_t)blockIdx.x * MAXT + t] + myrank;
    if (pos_of_atom) pos_of_atom[i] = pos;
    atom_of_pos[pos] = (int32_t)i;
  }
}

void launch_type_sort(hipStream_t s, int64_t n, const double4 *xw, int ntypes, int32_t *blk_counts,
                      int32_t *type_count, int32_t *type_start, int32_t *pos_of_atom, int32_t *atom_of_pos,
                      int64_t rows_cap, const int32_t *mask) {
  int nblk = (int)((n + TS_BLOCK - 1) / TS_BLOCK);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((rows_cap + 255) / 256)), dim3(256), 0, s, atom_of_pos, rows_cap,
                     -1);
  if (n <= 0) {
    hipLaunchKernelGGL(k_type_scan, dim3(1), dim3(64), 0, s, 0, ntypes, blk_counts, type_count, type_start);
    return;
  }
  hipLaunchKernelGGL(k_type_count, dim3(nblk), dim3(TS_BLOCK), 0, s, n, xw, ntypes, blk_counts, mask);
  hipLaunchKernelGGL(k_type_scan, dim3(1), dim3(64), 0, s, nblk, ntypes, blk_counts, type_count, type_start);
  hipLaunchKernelGGL(k_type_place, dim3(nblk), dim3(TS_BLOCK), 0, s, n, xw, ntypes, blk_counts, type_start,
                     pos_of_atom, atom_of_pos, mask);
}

// ---------------------------------------------------------------------------
// cell list: side >= rlist, counting sort by cell (order inside a cell is
// irrelevant: the formatted list is sorted by key afterwards)
// ---------------------------------------------------------------------------
__device__ inline int cell_coord(double x, double side, int nc) {
  int c = (int)floor(x / side);
  if (c >= nc) c = nc - 1;
  if (c < 0) c = 0;
  return c;
}

__device__ inline bool skip_build(const uint32_t *cond) { return cond && !(*cond & FLAG_REBUILD); }

__global__ void k_fill_cond(int32_t *p, int64_t n, int32_t v, const uint32_t *cond) {
  if (skip_build(cond)) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_cell_assign(int64_t n, const double4 *__restrict__ xw, CellGrid g, int32_t *cell_of,
                              int32_t *cell_count, const uint32_t *cond) {
  if (skip_build(cond)) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double4 p = xw[i];
  int cx = cell_coord(p.x, g.side[0], g.nc[0]);
  int cy = cell_coord(p.y, g.side[1], g.nc[1]);
  int cz = cell_coord(p.z, g.side[2], g.nc[2]);
  int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
  cell_of[i] = c;
  atomicAdd(&cell_count[c], 1);
}

// single-block exclusive scan of m int32 values: out[0..m] (out[m] = total)
__global__ void __launch_bounds__(1024) k_scan_single(const int32_t *in, int64_t m, int32_t *out,
                                                      const uint32_t *cond) {
  if (skip_build(cond)) return;
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < m; base += 1024) {
    int64_t i = base + threadIdx.x;
    int32_t v = (i < m) ? in[i] : 0;
    int32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      int32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int32_t woff = 0;
    for (int w = 0; w < wv; ++w) woff += wsum[w];
    int32_t c0 = carry;
    if (i < m) out[i] = c0 + woff + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = c0 + woff + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = carry;
}

// code[i] = cx << 24 | cy << 16 | cz << 8 | min(index inside the cell, 255)
// (cell coordinates modulo 256; used only with at most 255 cells per axis)
__global__ void k_cell_fill(int64_t n, CellGrid g, const int32_t *cell_of, const int32_t *cell_start,
                            int32_t *cell_fill, int32_t *cell_atoms, uint32_t *code, const uint32_t *cond) {
  if (skip_build(cond)) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_of[i];
  int p = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + p] = (int32_t)i;
  if (code) {
    const int cz = c % g.nc[2], cy = (c / g.nc[2]) % g.nc[1], cx = c / (g.nc[1] * g.nc[2]);
    code[i] = ((uint32_t)(cx & 255) << 24) | ((uint32_t)(cy & 255) << 16) | ((uint32_t)(cz & 255) << 8) |
              (uint32_t)(p < 255 ? p : 255);
  }
}

void launch_cells(hipStream_t s, int64_t n, const double4 *xw, const CellGrid &g, int32_t *cell_of,
                  int32_t *cell_start, int32_t *cell_fill, int32_t *cell_atoms, uint32_t *cell_code,
                  int32_t *scan_tmp, const uint32_t *cond) {
  int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
  unsigned gc = (unsigned)((ncell + 255) / 256);
  hipLaunchKernelGGL(k_fill_cond, dim3(gc), dim3(256), 0, s, scan_tmp, ncell, 0, cond);
  hipLaunchKernelGGL(k_fill_cond, dim3(gc), dim3(256), 0, s, cell_fill, ncell, 0, cond);
  if (n > 0)
    hipLaunchKernelGGL(k_cell_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, xw, g, cell_of,
                       scan_tmp, cond);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, scan_tmp, ncell, cell_start, cond);
  if (n > 0)
    hipLaunchKernelGGL(k_cell_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, g, cell_of,
                       cell_start, cell_fill, cell_atoms, cell_code, cond);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

// ---------------------------------------------------------------------------
// candidates within rlist (= rc + skin, slightly inflated so that the exact
// r <= rc test of the formatting kernel only ever removes pairs): one wave
// per atom, lanes stride over the atoms of each adjacent cell.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_candidates(int64_t n, const double4 *__restrict__ xw, CellGrid g,
                                                    const int32_t *__restrict__ cell_start,
                                                    const int32_t *__restrict__ cell_atoms, double rl2, int cap,
                                                    int32_t *__restrict__ cand, int32_t *__restrict__ cand_n,
                                                    uint32_t *flags, const uint32_t *cond) {
  if (skip_build(cond)) return;
  int lane = threadIdx.x & 63;
  int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double4 p = xw[i];
  int c0[3] = {cell_coord(p.x, g.side[0], g.nc[0]), cell_coord(p.y, g.side[1], g.nc[1]),
               cell_coord(p.z, g.side[2], g.nc[2])};
  int offs[3][3], no[3];
  for (int a = 0; a < 3; ++a) {
    int cnt = 0;
    for (int t = -1; t <= 1; ++t) {
      int v = ((c0[a] + t) % g.nc[a] + g.nc[a]) % g.nc[a];
      bool dup = false;
      for (int q = 0; q < cnt; ++q) dup |= (offs[a][q] == v);
      if (!dup) offs[a][cnt++] = v;
    }
    no[a] = cnt;
  }
  int32_t count = 0;
  int32_t *out = cand + i * (int64_t)cap;
  for (int ax = 0; ax < no[0]; ++ax)
    for (int ay = 0; ay < no[1]; ++ay)
      for (int az = 0; az < no[2]; ++az) {
        int c = (offs[0][ax] * g.nc[1] + offs[1][ay]) * g.nc[2] + offs[2][az];
        int b = cell_start[c], e = cell_start[c + 1];
        for (int q = b; q < e; q += 64) {
          bool keep = false;
          int32_t j = -1;
          if (q + lane < e) {
            j = cell_atoms[q + lane];
            if (j != i) {
              double4 pj = xw[j];
              double dx = min_image(pj.x - p.x, g.L[0]);
              double dy = min_image(pj.y - p.y, g.L[1]);
              double dz = min_image(pj.z - p.z, g.L[2]);
              double r2 = dx * dx + dy * dy;
              r2 = r2 + dz * dz;
              keep = r2 <= rl2;
            }
          }
          unsigned long long m = __ballot(keep);
          int pre = __popcll(m & ((1ull << lane) - 1ull));
          if (keep && count + pre < cap) out[count + pre] = j;
          count += __popcll(m);
        }
      }
  if (lane == 0) {
    cand_n[i] = count < cap ? count : cap;
    if (count > cap) atomicOr(flags, FLAG_CAND_CAP);
  }
}

void launch_candidates(hipStream_t s, int64_t n, const double4 *xw, const CellGrid &g, const int32_t *cell_start,
                       const int32_t *cell_atoms, double rlist, int cand_cap, int32_t *cand, int32_t *cand_n,
                       uint32_t *flags, const uint32_t *cond) {
  if (n <= 0) return;
  double rl2 = rlist * rlist * (1.0 + 1e-9);
  hipLaunchKernelGGL(k_candidates, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, xw, g, cell_start,
                     cell_atoms, rl2, cand_cap, cand, cand_n, flags, cond);
}

// ---------------------------------------------------------------------------
// formatting (Section V-B): one wave per atom, keys in LDS.  The keys are
// ranked exactly by a bucketed counting sort: bucket = type * FMT_NB +
// floor(FMT_NB (quantised distance / (quantised rc + 1))^3), monotone in the
// key and holding equal expected counts (neighbours grow like r^3), so
// rank = (keys in lower buckets, from a prefix scan of the bucket
// histogram) + (smaller keys of the same bucket, from the bucket's linked
// list in LDS).
// ---------------------------------------------------------------------------
constexpr int FMT_WAVES = 4;
constexpr int FMT_CAP = KEY_CAP;
constexpr int FMT_NB = 64;   // distance buckets per type

// bucket of a key with type t and quantised distance qd < qlim (inv_qlim =
// 1 / qlim in FP32); monotone non-decreasing in (t, qd) (every step is), the
// same expression at insertion and at ranking
__device__ inline int fmt_bucket(int t, unsigned long long qd, float inv_qlim) {
  const float x = (float)qd * inv_qlim;
  const int b = (int)(x * x * x * (float)FMT_NB);
  return t * FMT_NB + (b < FMT_NB - 1 ? b : FMT_NB - 1);
}
constexpr int FMT_BATCH = 4; // candidate gathers in flight per lane

// per-wave LDS of the format kernel: keys (staged r^2 first) [FMT_CAP] u64,
// neighbour and type [FMT_CAP] i32, bucket heads and starts [nb] i32 each,
// list links [FMT_CAP] i16
__host__ __device__ inline size_t fmt_wave_bytes(int nb) {
  return (size_t)FMT_CAP * 8 + (size_t)FMT_CAP * 4 + (size_t)nb * 8 + (size_t)FMT_CAP * 2;
}

__global__ void __launch_bounds__(256) k_format(int64_t n, const double4 *__restrict__ xw, Dims d, double L0,
                                                double L1, double L2, double rc2max,
                                                const int32_t *__restrict__ cand,
                                                const int32_t *__restrict__ cand_n, int cap,
                                                int32_t *__restrict__ nlist, int32_t *__restrict__ nreal,
                                                unsigned long long *overflow, int32_t *max_real, uint32_t *flags,
                                                float4 *__restrict__ rt32) {
  extern __shared__ __align__(16) unsigned char fmt_lds[];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t i = (int64_t)blockIdx.x * FMT_WAVES + wv;
  if (i >= n) return;
  const int nb_tot = d.ntypes * FMT_NB;
  unsigned char *wb = fmt_lds + (size_t)wv * fmt_wave_bytes(nb_tot);
  unsigned long long *keys = (unsigned long long *)wb;
  int32_t *jt = (int32_t *)(wb + (size_t)FMT_CAP * 8);
  int32_t *head = jt + FMT_CAP;
  int32_t *bstart = head + nb_tot;
  int16_t *next = (int16_t *)(bstart + nb_tot);
  const unsigned long long below = (1ull << lane) - 1ull;
  // keys stored and neighbours within rc per type, wave-uniform: ballot
  // prefix counts instead of atomics on one LDS address
  int kc = 0;
  int tc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) tc[t] = 0;
  for (int b = lane; b < nb_tot; b += 64) {
    head[b] = -1;
    bstart[b] = 0;
  }
  const double inv_w = 1.0 / (d.rcut - d.rcut_smth);
  const unsigned long long qlim = (unsigned long long)floor(d.rcut * 1e8) + 1ull;
  const float inv_qlim = 1.0f / (float)qlim;
  double4 p = xw[i];
  int nc = cand_n[i];
  const int32_t *ci = cand + i * (int64_t)cap;
  // pass 1: distances of all candidates; those within rc (r^2 <= rc2max,
  // the largest double whose square root is <= rc, so the same test as
  // sqrt(r^2) <= rc) are staged compactly, r^2 in their key slot
  for (int q0 = 0; q0 < nc; q0 += 64 * FMT_BATCH) {
    // issue the index loads, then the position gathers, of FMT_BATCH rounds
    // unconditional loads (lanes past the list reread its last entry and
    // are then masked), so none of them waits behind a branch
    int32_t jb[FMT_BATCH];
    double4 pb[FMT_BATCH];
#pragma unroll
    for (int u = 0; u < FMT_BATCH; ++u) {
      const int q = q0 + 64 * u + lane;
      jb[u] = ci[q < nc ? q : nc - 1];
    }
#pragma unroll
    for (int u = 0; u < FMT_BATCH; ++u) pb[u] = xw[jb[u]];
#pragma unroll
    for (int u = 0; u < FMT_BATCH; ++u)
      if (q0 + 64 * u + lane >= nc) {
        jb[u] = -1;
        pb[u] = p;
      }
#pragma unroll
    for (int u = 0; u < FMT_BATCH; ++u) {
      const int32_t j = jb[u];
      const double4 pj = pb[u];  // = p for lanes without a candidate (r = 0, not kept)
      double dx = min_image(pj.x - p.x, L0);
      double dy = min_image(pj.y - p.y, L1);
      double dz = min_image(pj.z - p.z, L2);
      double r2 = dx * dx + dy * dy;
      r2 = r2 + dz * dz;
      const bool keep = j >= 0 && r2 <= rc2max;
      const unsigned long long m = __ballot(keep);
      if (m == 0ull) continue;
      const int tj = (int)pj.w;
      const int slot = kc + __popcll(m & below);
      kc += __popcll(m);
#pragma unroll
      for (int t = 0; t < MAXT; ++t)
        if (t < d.ntypes) tc[t] += __popcll(__ballot(keep && tj == t));
      if (keep && slot < FMT_CAP) {
        keys[slot] = (unsigned long long)__double_as_longlong(r2);
        jt[slot] = j | (tj << 26);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int k = kc;
  if (k > FMT_CAP) {
    if (lane == 0) atomicOr(flags, FLAG_KEY_CAP);
    k = FMT_CAP;
  }
  // pass 2, dense over the lanes: r, the key (type, floor(r 1e8), index)
  // and its bucket's linked list
  for (int q = lane; q < k; q += 64) {
    const double r = sqrt(__longlong_as_double((long long)keys[q]));
    const int32_t v = jt[q];
    const unsigned long long tj = (unsigned long long)(v >> 26), j = (unsigned long long)(v & ((1 << 26) - 1));
    const unsigned long long qd = (unsigned long long)floor(r * 1e8);
    keys[q] = (tj << 58) | (qd << 26) | j;
    const int b = fmt_bucket((int)tj, qd, inv_qlim);
    next[q] = (int16_t)atomicExch(&head[b], q);
    atomicAdd(&bstart[b], 1);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // exclusive scan of the bucket histogram: lane takes a run of buckets
  {
    const int per = (nb_tot + 63) / 64;
    const int b0 = lane * per;
    int run = 0;
    for (int b = b0; b < b0 + per && b < nb_tot; ++b) run += bstart[b];
    int incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    int acc = incl - run;
    for (int b = b0; b < b0 + per && b < nb_tot; ++b) {
      const int c = bstart[b];
      bstart[b] = acc;
      acc += c;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int tstart[MAXT], treal[MAXT];
  {
    int run = 0;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int c = t < d.ntypes ? tc[t] : 0;
      tstart[t] = run;
      run += c;
      treal[t] = t < d.ntypes ? (c < d.sel[t] ? c : d.sel[t]) : 0;
    }
  }
  int32_t *row = nlist + i * (int64_t)d.nnei;
  // exact rank of each key (keys are distinct)
  for (int q = lane; q < k; q += 64) {
    const unsigned long long key = keys[q];
    const int t = (int)(key >> 58);
    const int b = fmt_bucket(t, (key >> 26) & 0xffffffffull, inv_qlim);
    int rank = bstart[b];
    for (int m = head[b]; m >= 0; m = next[m]) rank += (keys[m] < key) ? 1 : 0;
    int ts = 0;
#pragma unroll
    for (int u = 0; u < MAXT; ++u)
      if (u == t) ts = tstart[u];
    int pos = rank - ts;
    // pos < 0 can only happen when the key buffer overflowed (flagged above)
    if (pos >= 0 && pos < d.sel[t]) {
      const int32_t j = (int32_t)(key & ((1ull << 26) - 1ull));
      row[d.off[t] + pos] = j;
      if (rt32) {
        // the slot's environment row (the mixed path's FP32 copy of FP64
        // values: from 1/r = rsqrt(r^2) with two Newton steps instead of the
        // environment kernel's square root and divisions, within an ulp or
        // two of its values before the rounding to FP32)
        const double4 D = pair_disp_sq(p, xw[j], L0, L1, L2);
        const double ir = rsqrt64(D.w), r = D.w * ir;
        const double x = fmin(fmax((r - d.rcut_smth) * inv_w, 0.0), 1.0);
        const double sv = (x * x * x * (-6.0 * x * x + 15.0 * x - 10.0) + 1.0) * ir, tv = sv * ir;
        rt32[i * (int64_t)d.nnei + d.off[t] + pos] =
            make_float4((float)sv, (float)(tv * D.x), (float)(tv * D.y), (float)(tv * D.z));
      }
    }
  }
  // only the real slots are written; k_pad_nlist fills the -1 padding when
  // the list is copied out (every device consumer stops at the real count)
  if (lane < d.ntypes) {
    int c = 0, cr = 0;
#pragma unroll
    for (int t = 0; t < MAXT; ++t)
      if (t == lane) {
        c = tc[t];
        cr = treal[t];
      }
    nreal[i * d.ntypes + lane] = cr;
    // the maximum only grows during the launch, so a stale read can only
    // cost an extra atomic; skipping the rest keeps 500k waves from
    // serialising on one address
    if (c > __hip_atomic_load(&max_real[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&max_real[lane], c);
    if (c > d.sel[lane]) atomicAdd(overflow, (unsigned long long)(c - d.sel[lane]));
  }
}

void launch_format(hipStream_t s, int64_t n, const double4 *xw, const Dims &d, const double *L, const int32_t *cand,
                   const int32_t *cand_n, int cand_cap, int32_t *nlist, int32_t *nreal, unsigned long long *overflow,
                   int32_t *max_real, uint32_t *flags, float4 *rt32) {
  if (n <= 0) return;
  // the largest double x with sqrt(x) <= rc (sqrt is correctly rounded and
  // monotone, so r^2 <= x exactly when sqrt(r^2) <= rc)
  double x = d.rcut * d.rcut;
  while (std::sqrt(x) > d.rcut) x = std::nextafter(x, 0.0);
  while (std::sqrt(std::nextafter(x, HUGE_VAL)) <= d.rcut) x = std::nextafter(x, HUGE_VAL);
  const size_t lds = FMT_WAVES * fmt_wave_bytes(d.ntypes * FMT_NB);
  hipLaunchKernelGGL(k_format, dim3((unsigned)((n + FMT_WAVES - 1) / FMT_WAVES)), dim3(64 * FMT_WAVES), lds, s, n, xw,
                     d, L[0], L[1], L[2], x, cand, cand_n, cand_cap, nlist, nreal, overflow, max_real, flags, rt32);
}

// -1 in every slot past a type's real count
__global__ void k_pad_nlist(int64_t n, Dims d, const int32_t *__restrict__ nreal, int32_t *__restrict__ nlist) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  for (int t = 0; t < d.ntypes; ++t) {
    const int r = nreal[i * d.ntypes + t];
    for (int sl = r + lane; sl < d.sel[t]; sl += 64) nlist[i * (int64_t)d.nnei + d.off[t] + sl] = -1;
  }
}

void launch_pad_nlist(hipStream_t s, int64_t n, const Dims &d, const int32_t *nreal, int32_t *nlist) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pad_nlist, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, d, nreal, nlist);
}

// ---------------------------------------------------------------------------
// skin check and reference copy for the MD driver
// ---------------------------------------------------------------------------
__global__ void k_max_disp(int64_t n, const double4 *__restrict__ xw, const double4 *__restrict__ xref, double L0,
                           double L1, double L2, double hs2, uint32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool far = false;
  if (i < n) {
    double4 a = xw[i], b = xref[i];
    double dx = min_image(a.x - b.x, L0), dy = min_image(a.y - b.y, L1), dz = min_image(a.z - b.z, L2);
    far = dx * dx + dy * dy + dz * dz > hs2;
  }
  if (__ballot(far) && (threadIdx.x & 63) == 0) atomicOr(flags, FLAG_REBUILD);
}

void launch_max_disp(hipStream_t s, int64_t n, const double4 *xw, const double4 *xref, const double *L,
                     double half_skin, uint32_t *flags) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_max_disp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, xw, xref, L[0], L[1], L[2],
                     half_skin * half_skin, flags);
}

__global__ void k_copy_ref(int64_t n, const double4 *__restrict__ xw, double4 *__restrict__ xref,
                           const uint32_t *cond) {
  if (skip_build(cond)) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) xref[i] = xw[i];
}

void launch_copy_ref(hipStream_t s, int64_t n, const double4 *xw, double4 *xref, const uint32_t *cond) {
  if (n > 0)
    hipLaunchKernelGGL(k_copy_ref, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, xw, xref, cond);
}

__global__ void k_end_rebuild(uint32_t *flags, unsigned long long *nbuild) {
  if (threadIdx.x == 0 && (*flags & FLAG_REBUILD)) {
    *flags &= ~FLAG_REBUILD;
    *nbuild += 1ull;
  }
}

void launch_end_rebuild(hipStream_t s, uint32_t *flags, unsigned long long *nbuild) {
  hipLaunchKernelGGL(k_end_rebuild, dim3(1), dim3(64), 0, s, flags, nbuild);
}

}  // namespace dpk
