// Declarations of the student embedding-net kernels (k_student.hip): a
// smaller net 1 -> 16 -> 32 -> M1 (tanh, doubling-skip tanh, affine output)
// fitted to the teacher's G(s) on neighbour distances of the current
// configuration.  Not part of the public ABI.
#pragma once
#include "dp_internal.h"

namespace dpk {

constexpr int SH1 = 16, SH2 = 32;  // student hidden widths
constexpr int SNF = SH2 + 1;       // features of the output-layer least squares (h2, 1)
constexpr int ST_ATTEMPTS = 32;    // rejection-sampling attempts per sample

// FP32 training parameters of one net, packed: W1[16] b1[16] W2[16][32]
// b2[32] W3[32][M1] b3[M1] (row = input feature).
struct StudentLayout {
  int o_w1, o_b1, o_w2, o_b2, o_w3, o_b3, np;
};
__host__ __device__ inline StudentLayout student_layout(int M1) {
  StudentLayout L;
  L.o_w1 = 0;
  L.o_b1 = SH1;
  L.o_w2 = 2 * SH1;
  L.o_b2 = L.o_w2 + SH1 * SH2;
  L.o_w3 = L.o_b2 + SH2;
  L.o_b3 = L.o_w3 + SH2 * M1;
  L.np = L.o_b3 + M1;
  return L;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based
// generator: output number `ctr` (0-based) of the stream seeded with `seed`.
__host__ __device__ inline uint64_t sm64(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1ull) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
// counter of attempt a of sample q of net `net`
__host__ __device__ inline uint64_t st_ctr(int net, int64_t q, int a) {
  return ((((uint64_t)net) << 40) + (uint64_t)q) * (uint64_t)ST_ATTEMPTS + (uint64_t)a;
}

struct StSampleArgs {
  Dims d;                      // teacher dims: ntypes, sel, off, nnei
  const int32_t *type_count;   // [ntypes]
  const int32_t *type_start;   // [ntypes] first type-sorted position
  const int32_t *atom_of_pos;  // [rows]
  const int32_t *nreal;        // [natoms][ntypes]
  const double4 *xw;           // [natoms] wrapped positions (s = sw(r) / r is recomputed)
  const int32_t *nlist;        // [natoms][nnei]
  double L[3];                 // box lengths
  uint64_t seed;
  int64_t q0;                  // index of the first batch's first sample
  int batch;                   // samples per net and batch
  int nb;                      // consecutive batches drawn (sample indices q0 .. q0 + nb * batch - 1)
  double *s;                   // [nb][nets][batch]
  float *wt;                   // [nb][nets][batch] 1 = drawn, 0 = no neighbour found
};
void launch_st_sample(hipStream_t st, const StSampleArgs &a);

struct StTeacherArgs {
  Dims d;                      // teacher embedding dims
  EmbOffsets eo;
  const double *ew;            // teacher FP64 padded weights
  int batch;
  int nb;                      // batches, as drawn by the sampler
  const double *s;             // [nb][nets][batch]
  double *G;                   // [nb][nets][batch][M1]
};
void launch_st_teacher(hipStream_t st, const StTeacherArgs &a);

struct StGradArgs {
  int M1, nets, batch;         // batch is a multiple of 64
  const float *params;         // [nets][np]
  const double *s;
  const float *wt;
  const double *G;
  float *gpart;                // [nets][batch/64][np] sums of r dG/dtheta
  double *lpart;               // [nets][batch/64][2]: sum of r^2, sum of weights
};
void launch_st_grad(hipStream_t st, const StGradArgs &a);

struct StAdamArgs {
  int M1, nets, nblk;
  float *params, *m, *v;
  const float *gpart;
  const double *lpart;
  float lr, b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
  double *loss;                // [nets] mean squared error of the batch
  float *g_out;                // when set: write the gradient, do not update
};
void launch_st_adam(hipStream_t st, const StAdamArgs &a);

struct StLsArgs {
  int M1, nets, batch, nblk;   // nblk blocks per net share the samples
  int nb;                      // batches of the draw ([nb][nets][batch] layout)
  const float *params;
  int quant;                   // -1 exact, 0 FP16, 1 BF16 rounding of W2
  const double *s;
  const float *wt;
  const double *G;
  double *part;                // [nets][nblk][SNF*SNF + SNF*M1], accumulated
};
void launch_st_ls(hipStream_t st, const StLsArgs &a);
int st_ls_blocks();
constexpr int ST_LS_FOLD = 32;  // slices the least-squares partials are folded into before the solve
// fold[net][slice][e] = sum of part[net][b][e] over the slice's blocks b (nblk % ST_LS_FOLD == 0)
void launch_st_lsfold(hipStream_t st, int M1, int nets, int nblk, const double *part, double *fold);

struct StSolveArgs {
  int M1, nets, nblk;
  const double *part;
  double ridge;                // relative to trace/SNF
  int quant;                   // -1 exact, 0 FP16, 1 BF16 rounding of W3
  double *X;                   // [nets][SNF][M1]: rows 0..31 W3, row 32 b3
  int32_t *status;             // [nets] 0 ok, 1 not positive definite, 2 no samples
};
void launch_st_solve(hipStream_t st, const StSolveArgs &a);

struct StCheckArgs {
  int M1, nets, batch;
  const float *params;
  const double *X;
  int quant;
  const double *s;
  const float *wt;
  const double *G;
  double *part;                // [nets][batch/64][2]: sum err^2, sum G^2
};
void launch_st_check(hipStream_t st, const StCheckArgs &a);

// force RMSE between two force arrays: part[grid] partial sums, out[0] = sqrt(mean |dF|^2)
void launch_force_rmse(hipStream_t st, const double *fa, const double *fb, int64_t n, double *part, double *out);

// sampled judge: mark[i] = 2 inside the cube of half side h around c
// (minimum image, per axis), 1 inside the cube of half side hr, else 0
void launch_judge_mark(hipStream_t st, int64_t n, const double4 *xw, const double *c, const double *L, double h,
                       double hr, int32_t *mark);
// force RMSE over the atoms with mark == 2; part needs 2 * 256 doubles
void launch_force_rmse_masked(hipStream_t st, const double *fa, const double *fb, int64_t n, const int32_t *mark,
                              double *part, double *out, double *count);
void launch_copy_i32(hipStream_t st, const int32_t *src, int32_t *dst);

// 16-bit rounding (round to nearest even) of a float, back as double
__host__ __device__ inline double st_round16(float x, int quant) {
  if (quant == 0) return (double)(float)(_Float16)x;
  if (quant == 1) {
    union {
      float f;
      uint32_t u;
    } v;
    v.f = x;
    v.u += 0x7fffu + ((v.u >> 16) & 1u);
    v.u &= 0xffff0000u;
    return (double)v.f;
  }
  return (double)x;
}

}  // namespace dpk
