// Student embedding net: sampling, teacher targets, training and the
// output-layer least squares.
//
// The student is a smaller embedding net, 1 -> 16 (tanh) -> 32 (tanh with
// the doubling skip) -> M1 (affine), one per (centre type, neighbour type)
// pair like the teacher's.  It is fitted to the teacher's own G(s) at
// neighbour distances of the current configuration:
//   1. samples: uniform over the real (centre, neighbour) pairs of each
//      type pair, by rejection (random centre of type t, random slot below
//      sel_u, kept when the slot holds a real neighbour), with SplitMix64 as
//      a counter-based generator so that every sample has a fixed identity;
//   2. targets: the teacher's G(s) in FP64;
//   3. Adam (Kingma and Ba, 2015) on the mean squared error in FP32;
//   4. the exact minimiser of the same squared error over the affine output
//      layer given the trained hidden layers: FP64 normal equations of
//      (h2, 1) with a small ridge, solved by Cholesky.  When the student will
//      run in 16-bit precision, W2 is rounded before the features are formed
//      and W3 after the solve, and b3 then absorbs the mean residual.
// Training work is small next to an MD run, so these kernels are plain
// FP32/FP64 VALU code with LDS; they spread each sample over several threads
// so that a batch of a few thousand samples still fills the chip.
#include "dp_f64.h"
#include "dp_student.h"

namespace dpk {

// ---------------------------------------------------------------------------
// 1. samples
// ---------------------------------------------------------------------------
__global__ void k_st_sample(StSampleArgs a) {
  const int net = blockIdx.y;
  const int T = a.d.ntypes;
  const int64_t nbk = blockIdx.z;  // batch of the draw
  const int t = net / T, u = net % T;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.batch) return;
  const int64_t count = a.type_count[t];
  const int64_t selu = a.d.sel[u];
  double s = 0.0;
  float w = 0.f;
  if (count > 0 && selu > 0) {
    for (int at = 0; at < ST_ATTEMPTS; ++at) {
      const uint64_t x = sm64(a.seed, st_ctr(net, a.q0 + nbk * a.batch + q, at));
      const int64_t k = (int64_t)(((x >> 32) * (uint64_t)count) >> 32);
      const int64_t slot = (int64_t)(((x & 0xffffffffull) * (uint64_t)selu) >> 32);
      const int i = a.atom_of_pos[a.type_start[t] + k];
      if (slot < a.nreal[(int64_t)i * T + u]) {
        const int j = a.nlist[(int64_t)i * a.d.nnei + a.d.off[u] + slot];
        const double4 D = pair_disp(a.xw[i], a.xw[j], a.L[0], a.L[1], a.L[2]);
        s = env_s(D.w, a.d.rcut_smth, a.d.rcut, 1.0 / (a.d.rcut - a.d.rcut_smth));
        w = 1.f;
        break;
      }
    }
  }
  const int64_t o = (nbk * T * T + net) * a.batch + q;
  a.s[o] = s;
  a.wt[o] = w;
}

void launch_st_sample(hipStream_t st, const StSampleArgs &a) {
  const int nets = a.d.ntypes * a.d.ntypes;
  hipLaunchKernelGGL(k_st_sample, dim3((a.batch + 255) / 256, nets, a.nb), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// 2. teacher G(s) in FP64 on the matrix cores: a wave takes 16 samples (the
//    MFMA N dimension); layer 0 on the VALU into a per-wave LDS tile
//    [feature][sample], each later layer as W^T H^T four output tiles at a
//    time (the embedding kernels' layer code), the last layer's outputs
//    written straight to G
// ---------------------------------------------------------------------------
constexpr int TCH_WAVES = 4;

// rows of the two per-wave activation buffers (outputs of the hidden layers
// l < n_emb - 1, layer l into buffer l & 1)
static void tch_rows(const Dims &d, int &r0, int &r1) {
  r0 = r1 = 0;
  for (int l = 0; l < d.n_emb - 1; ++l) {
    int &r = (l & 1) ? r1 : r0;
    r = d.ekp[l + 1] > r ? d.ekp[l + 1] : r;
  }
}

__global__ void __launch_bounds__(64 * TCH_WAVES) k_st_teacher(StTeacherArgs a, int r0, int r1) {
  extern __shared__ double tsh[];
  const Dims &d = a.d;
  const int net = blockIdx.y;
  const int t = net / d.ntypes, u = net % d.ntypes;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = lane & 15;
  const int q0 = (blockIdx.x * TCH_WAVES + wv) * 16;
  if (q0 >= a.batch) return;  // the whole wave
  const int64_t row = ((int64_t)blockIdx.z * d.ntypes * d.ntypes + net) * a.batch;  // first sample of (batch, net)
  double *buf[2] = {tsh + (size_t)wv * (r0 + r1) * 16, tsh + (size_t)wv * (r0 + r1) * 16 + r0 * 16};
  // unconditional load: samples past the batch reread its last one and are not written
  const double s = a.s[row + (q0 + n < a.batch ? q0 + n : a.batch - 1)];
  {
    const double *W0 = a.ew + a.eo.w[t][u][0], *b0 = a.ew + a.eo.b[t][u][0];
    const int out = d.ew[1];
    for (int idx = lane; idx < d.ekp[1] * 16; idx += 64) {
      const int f = idx >> 4;  // sample idx & 15 == n
      double h = 0.0;
      if (f < out) {
        h = tanh64(s * W0[f] + b0[f]);
        if (out <= 2) h += s;  // identity / doubling skip of the scalar input
      }
      buf[0][f * 16 + n] = h;
    }
  }
  wave_sync();
  for (int l = 1; l < d.n_emb; ++l) {
    const int in = d.ew[l], out = d.ew[l + 1];
    const bool last = l == d.n_emb - 1;
    const bool lin = d.emb_lin && last;
    const double *Hin = buf[(l - 1) & 1];
    double *Hout = buf[l & 1];
    const int rows_out = last ? 0 : d.ekp[l + 1];
    const double *W = a.ew + a.eo.w[t][u][l], *bias = a.ew + a.eo.b[t][u][l];
    const int nmt = d.emp[l + 1] >> 4;
    for (int mt0 = 0; mt0 < nmt; mt0 += EMB_G) {
      v4d acc[1][EMB_G];
      mfma_group<1>(W, d.ekp[l], d.emp[l + 1], Hin, 16, lane, mt0, acc);
#pragma unroll
      for (int g = 0; g < EMB_G; ++g) {
        const int mt = mt0 + g;
        if (mt >= nmt) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int f = mt * 16 + 4 * r + (lane >> 4);
          double h = 0.0;
          if (f < out) {
            const double z = acc[0][g][r] + bias[f];
            h = lin ? z : tanh64(z);
            const int sf = skip_src(f, in, out);
            if (sf >= 0) h += Hin[sf * 16 + n];
          }
          if (last) {
            if (f < out && q0 + n < a.batch) a.G[(row + q0 + n) * d.M1 + f] = h;
          } else if (f < rows_out) {
            Hout[f * 16 + n] = h;
          }
        }
      }
    }
    wave_sync();
  }
}

void launch_st_teacher(hipStream_t st, const StTeacherArgs &a) {
  int r0, r1;
  tch_rows(a.d, r0, r1);
  const size_t shm = (size_t)TCH_WAVES * (r0 + r1) * 16 * sizeof(double);
  const int nets = a.d.ntypes * a.d.ntypes;
  hipLaunchKernelGGL(k_st_teacher, dim3((a.batch + 16 * TCH_WAVES - 1) / (16 * TCH_WAVES), nets, a.nb),
                     dim3(64 * TCH_WAVES), shm, st, a, r0, r1);
}

// ---------------------------------------------------------------------------
// student forward in FP32 for one sample: h1, t1, h2, t2 in registers
// ---------------------------------------------------------------------------
constexpr int SP = 65;  // LDS row stride (samples), odd to spread banks

__device__ inline void st_hidden_f32(const float *P, const StudentLayout &L, float s, float (&t1)[SH1],
                                     float (&t2)[SH2], float (&h2)[SH2]) {
#pragma unroll
  for (int i = 0; i < SH1; ++i) t1[i] = tanhf(s * P[L.o_w1 + i] + P[L.o_b1 + i]);
#pragma unroll
  for (int j = 0; j < SH2; ++j) {
    float z = P[L.o_b2 + j];
#pragma unroll
    for (int i = 0; i < SH1; ++i) z += t1[i] * P[L.o_w2 + i * SH2 + j];
    t2[j] = tanhf(z);
    h2[j] = t1[j % SH1] + t2[j];
  }
}

// ---------------------------------------------------------------------------
// 3a. squared error and its gradient: GR_SPLIT blocks of eight waves per 64
//     samples; wave w takes output features [w*oc, (w+1)*oc) of every sample,
//     the partial dE/dh2 meet in LDS, and block z sums parameters
//     [z*per, (z+1)*per) over the 64 samples
// ---------------------------------------------------------------------------
constexpr int GR_WAVES = 8;
constexpr int GR_OC = 16;  // output features per wave at most (M1 <= 128)
// workgroups per 64 samples: each evaluates the samples and sums its share
// of the parameters (a 4,096-sample batch of one net is 64 x 4 workgroups)
constexpr int GR_SPLIT = 4;
constexpr int GSP = 68;  // LDS row stride of the gradient kernel (samples): 16-byte rows for float4 sums

__global__ void __launch_bounds__(64 * GR_WAVES) k_st_grad(StGradArgs a) {
  extern __shared__ float gsh[];
  const int M1 = a.M1;
  const StudentLayout L = student_layout(M1);
  const int net = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const int tid = threadIdx.x, m = tid & 63, wv = tid >> 6;
  float *P = gsh;                   // [np]
  float *ss = P + ((L.np + 3) & ~3); // [64], 16-byte aligned
  float *h1s = ss + 64;             // [SH1][GSP]
  float *dz1s = h1s + SH1 * GSP;     // [SH1][GSP]
  float *h2s = dz1s + SH1 * GSP;     // [SH2][GSP]
  float *dz2s = h2s + SH2 * GSP;     // [SH2][GSP]
  float *rs = dz2s + SH2 * GSP;      // [M1][GSP]
  float *dhp = rs + M1 * GSP;        // [GR_WAVES][SH2][GSP] partial dE/dh2
  __shared__ double red[2][64 * GR_WAVES];
  const float *Pg = a.params + (int64_t)net * L.np;
  for (int e = tid; e < L.np; e += 64 * GR_WAVES) P[e] = Pg[e];
  __syncthreads();
  const int64_t q = (int64_t)net * a.batch + (int64_t)blk * 64 + m;
  const float s = (float)a.s[q];
  const float w = a.wt[q];
  static_assert(SH1 == 2 * GR_WAVES && SH2 == 4 * GR_WAVES, "hidden features split evenly over the waves");
  // forward, each hidden feature once per sample: wave wv takes the first
  // layer's features 2 wv, 2 wv + 1 and the second layer's 4 wv .. 4 wv + 3
  // (the same expressions as st_hidden_f32), shared through LDS
  float t1o[2], t2o[4];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int i = 2 * wv + c;
    t1o[c] = tanhf(s * P[L.o_w1 + i] + P[L.o_b1 + i]);
    h1s[i * GSP + m] = t1o[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = 4 * wv + c;
    float z = P[L.o_b2 + j];
#pragma unroll
    for (int i = 0; i < SH1; ++i) z += h1s[i * GSP + m] * P[L.o_w2 + i * SH2 + j];
    t2o[c] = tanhf(z);
    h2s[j * GSP + m] = h1s[(j % SH1) * GSP + m] + t2o[c];
  }
  __syncthreads();
  float h2[SH2];
#pragma unroll
  for (int j = 0; j < SH2; ++j) h2[j] = h2s[j * GSP + m];
  float dh2[SH2];
#pragma unroll
  for (int k = 0; k < SH2; ++k) dh2[k] = 0.f;
  double lsum = 0.0;
  const double *Gt = a.G + q * M1;
  const int oc = (M1 + GR_WAVES - 1) / GR_WAVES;  // <= GR_OC (M1 <= 128)
  const int o0 = wv * oc, o1 = o0 + oc < M1 ? o0 + oc : M1;
  // this wave's teacher targets, all loads issued before the first use
  // (unconditional: indices past the range reread the last output)
  double gt[GR_OC];
#pragma unroll
  for (int k = 0; k < GR_OC; ++k) gt[k] = Gt[o0 + k < M1 ? o0 + k : M1 - 1];
#pragma unroll
  for (int k = 0; k < GR_OC; ++k) {
    const int o = o0 + k;
    if (o >= o1) break;
    float g = P[L.o_b3 + o];
#pragma unroll
    for (int j = 0; j < SH2; ++j) g += h2[j] * P[L.o_w3 + j * M1 + o];
    const float r = w * (g - (float)gt[k]);
    lsum += (double)r * r;
    rs[o * GSP + m] = r;
#pragma unroll
    for (int j = 0; j < SH2; ++j) dh2[j] += P[L.o_w3 + j * M1 + o] * r;
  }
#pragma unroll
  for (int k = 0; k < SH2; ++k) dhp[(wv * SH2 + k) * GSP + m] = dh2[k];
  red[0][tid] = lsum;
  red[1][tid] = wv == 0 ? (double)w : 0.0;
  __syncthreads();
  // backward through the hidden layers, split over the waves as the forward:
  // dE/dh2 summed over the waves' partials in wave order, then
  // dz2 = dE/dh2 (1 - t2^2) (into the wave-0 slice of the partials, which
  // only this wave reads), then dz1 from all of dz2
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int k = 4 * wv + c;
    float v = 0.f;
#pragma unroll
    for (int w2 = 0; w2 < GR_WAVES; ++w2) v += dhp[(w2 * SH2 + k) * GSP + m];
    dhp[k * GSP + m] = v;  // dE/dh2
    dz2s[k * GSP + m] = v * (1.f - t2o[c] * t2o[c]);
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int i = 2 * wv + c;
    float g = dhp[i * GSP + m] + dhp[(i + SH1) * GSP + m];
#pragma unroll
    for (int j = 0; j < SH2; ++j) g += P[L.o_w2 + i * SH2 + j] * dz2s[j * GSP + m];
    dz1s[i * GSP + m] = g * (1.f - t1o[c] * t1o[c]);
  }
  if (wv == 0) ss[m] = s;
  __syncthreads();
  // sums over the 64 samples of the block, parameter by parameter
  float *gp = a.gpart + ((int64_t)net * nblk + blk) * L.np;
  // 64-sample dot products and sums in float4 steps (rows are 16-byte aligned)
  auto dot64 = [](const float *x, const float *y) {
    float acc = 0.f;
#pragma unroll 4
    for (int k = 0; k < 64; k += 4) {
      const float4 u = *(const float4 *)(x + k), v = *(const float4 *)(y + k);
      acc += (u.x * v.x + u.y * v.y) + (u.z * v.z + u.w * v.w);
    }
    return acc;
  };
  auto sum64 = [](const float *x) {
    float acc = 0.f;
#pragma unroll 4
    for (int k = 0; k < 64; k += 4) {
      const float4 u = *(const float4 *)(x + k);
      acc += (u.x + u.y) + (u.z + u.w);
    }
    return acc;
  };
  // this block's share of the parameters (blockIdx.z of GR_SPLIT)
  const int per = (L.np + GR_SPLIT - 1) / GR_SPLIT;
  const int e_end = (int)blockIdx.z * per + per < L.np ? (int)blockIdx.z * per + per : L.np;
  for (int e = (int)blockIdx.z * per + tid; e < e_end; e += 64 * GR_WAVES) {
    float acc = 0.f;
    if (e < L.o_b1) {
      acc = dot64(ss, dz1s + e * GSP);
    } else if (e < L.o_w2) {
      acc = sum64(dz1s + (e - L.o_b1) * GSP);
    } else if (e < L.o_b2) {
      const int i = (e - L.o_w2) / SH2, j = (e - L.o_w2) % SH2;
      acc = dot64(h1s + i * GSP, dz2s + j * GSP);
    } else if (e < L.o_w3) {
      acc = sum64(dz2s + (e - L.o_b2) * GSP);
    } else if (e < L.o_b3) {
      const int kk = (e - L.o_w3) / M1, o = (e - L.o_w3) % M1;
      acc = dot64(h2s + kk * GSP, rs + o * GSP);
    } else {
      acc = sum64(rs + (e - L.o_b3) * GSP);
    }
    gp[e] = acc;
  }
  if (blockIdx.z == 0 && wv == 0) {
    // sums of the squared errors and of the weights: lane m takes every
    // 64th entry, then a butterfly over the wave
    double v0 = 0.0, v1 = 0.0;
    for (int k = m; k < 64 * GR_WAVES; k += 64) {
      v0 += red[0][k];
      v1 += red[1][k];
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      v0 += __shfl_xor(v0, o);
      v1 += __shfl_xor(v1, o);
    }
    if (m == 0) {
      a.lpart[((int64_t)net * nblk + blk) * 2 + 0] = v0;
      a.lpart[((int64_t)net * nblk + blk) * 2 + 1] = v1;
    }
  }
}

void launch_st_grad(hipStream_t st, const StGradArgs &a) {
  const StudentLayout L = student_layout(a.M1);
  const size_t shm =
      sizeof(float) * ((size_t)((L.np + 3) & ~3) + 64 + (size_t)(2 * SH1 + 2 * SH2 + a.M1 + GR_WAVES * SH2) * GSP);
  hipLaunchKernelGGL(k_st_grad, dim3(a.batch / 64, a.nets, GR_SPLIT), dim3(64 * GR_WAVES), shm, st, a);
}

// ---------------------------------------------------------------------------
// 3b. Adam: one thread per parameter; gradient = 2/(M1 sum w) sum r dG/dtheta
// ---------------------------------------------------------------------------
__global__ void k_st_adam(StAdamArgs a) {
  const StudentLayout L = student_layout(a.M1);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.nets * L.np) return;
  const int net = (int)(e / L.np), p = (int)(e % L.np);
  double wsum = 0.0, lsum = 0.0;
  float g = 0.f;
  // the partials in block order, sixteen loads in flight before their adds
  const int64_t pb0 = (int64_t)net * a.nblk;
  int b = 0;
  for (; b + 16 <= a.nblk; b += 16) {
    float gv[16];
    double lv[16], wv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      gv[u] = a.gpart[(pb0 + b + u) * L.np + p];
      lv[u] = a.lpart[(pb0 + b + u) * 2 + 0];
      wv[u] = a.lpart[(pb0 + b + u) * 2 + 1];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      g += gv[u];
      lsum += lv[u];
      wsum += wv[u];
    }
  }
  for (; b < a.nblk; ++b) {
    g += a.gpart[(pb0 + b) * L.np + p];
    lsum += a.lpart[(pb0 + b) * 2 + 0];
    wsum += a.lpart[(pb0 + b) * 2 + 1];
  }
  const double denom = (double)a.M1 * (wsum > 0.0 ? wsum : 1.0);
  g *= (float)(2.0 / denom);
  if (p == 0 && a.loss) a.loss[net] = lsum / denom;
  if (a.g_out) {
    a.g_out[e] = g;
    return;
  }
  const float m = a.b1 * a.m[e] + (1.f - a.b1) * g;
  const float v = a.b2 * a.v[e] + (1.f - a.b2) * g * g;
  a.m[e] = m;
  a.v[e] = v;
  a.params[e] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

void launch_st_adam(hipStream_t st, const StAdamArgs &a) {
  const StudentLayout L = student_layout(a.M1);
  const int64_t n = (int64_t)a.nets * L.np;
  hipLaunchKernelGGL(k_st_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
// 4a. normal equations of the output layer in FP64:
//     A = sum w phi phi^T (SNF x SNF), B = sum w phi G^T (SNF x M1),
//     phi = (h2(s), 1); each block accumulates its share into its partial
// ---------------------------------------------------------------------------
constexpr int LS_BLOCKS = 2048;  // enough 64-sample groups in flight for a whole draw
constexpr int LS_MAXE = (SNF * SNF + SNF * 128 + 63) / 64;  // entries per thread, M1 <= 128
static_assert(LS_BLOCKS % ST_LS_FOLD == 0, "the fold takes equal runs of blocks");
int st_ls_blocks() { return LS_BLOCKS; }

__device__ inline void st_hidden_f64(const float *P, const StudentLayout &L, int quant, double s,
                                     double (&h2)[SH2]) {
  double t1[SH1];
#pragma unroll
  for (int i = 0; i < SH1; ++i) t1[i] = tanh64(s * (double)P[L.o_w1 + i] + (double)P[L.o_b1 + i]);
#pragma unroll
  for (int j = 0; j < SH2; ++j) {
    double z = (double)P[L.o_b2 + j];
#pragma unroll
    for (int i = 0; i < SH1; ++i) z += t1[i] * st_round16(P[L.o_w2 + i * SH2 + j], quant);
    h2[j] = t1[j % SH1] + tanh64(z);
  }
}

__global__ void __launch_bounds__(64) k_st_ls(StLsArgs a) {
  extern __shared__ double lsh[];
  const int M1 = a.M1;
  const StudentLayout L = student_layout(M1);
  const int net = blockIdx.y, blk = blockIdx.x;
  const int tid = threadIdx.x;
  const int NE = SNF * SNF + SNF * M1;
  double *phi = lsh;             // [SNF][SP]
  double *gt = phi + SNF * SP;   // [M1][SP]
  const float *P = a.params + (int64_t)net * L.np;
  double acc[LS_MAXE];
#pragma unroll
  for (int k = 0; k < LS_MAXE; ++k) acc[k] = 0.0;
  const int gpb = a.batch / 64, ngroups = gpb * a.nb;  // 64-sample groups per batch, in the draw
  for (int gidx = blk; gidx < ngroups; gidx += a.nblk) {
    const int kb = gidx / gpb, gq = gidx % gpb;
    const int64_t q = ((int64_t)kb * a.nets + net) * a.batch + (int64_t)gq * 64 + tid;
    const double w = (double)a.wt[q];
    double h2[SH2];
    st_hidden_f64(P, L, a.quant, a.s[q], h2);
#pragma unroll
    for (int j = 0; j < SH2; ++j) phi[j * SP + tid] = w * h2[j];
    phi[SH2 * SP + tid] = w;
    const double *Gt = a.G + q * M1;
    for (int o = 0; o < M1; ++o) gt[o * SP + tid] = w * Gt[o];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LS_MAXE; ++k) {
      const int e = tid + 64 * k;
      if (e < NE) {
        const double *x, *y;
        if (e < SNF * SNF) {
          x = phi + (e / SNF) * SP;
          y = phi + (e % SNF) * SP;
        } else {
          const int e2 = e - SNF * SNF;
          x = phi + (e2 / M1) * SP;
          y = gt + (e2 % M1) * SP;
        }
        double v = 0.0;
        for (int m = 0; m < 64; ++m) v += x[m] * y[m];
        acc[k] += v;
      }
    }
    __syncthreads();
  }
  double *part = a.part + ((int64_t)net * a.nblk + blk) * NE;
#pragma unroll
  for (int k = 0; k < LS_MAXE; ++k) {
    const int e = tid + 64 * k;
    if (e < NE) part[e] += acc[k];
  }
}

void launch_st_ls(hipStream_t st, const StLsArgs &a) {
  const size_t shm = sizeof(double) * (size_t)(SNF + a.M1) * SP;
  hipLaunchKernelGGL(k_st_ls, dim3(a.nblk, a.nets), dim3(64), shm, st, a);
}

__global__ void k_st_lsfold(int NE, int nblk, const double *__restrict__ part, double *__restrict__ fold) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x, net = blockIdx.y, sl = blockIdx.z;
  if (e >= NE) return;
  const int per = nblk / ST_LS_FOLD;
  double v = 0.0;
  for (int b = sl * per; b < (sl + 1) * per; ++b) v += part[((int64_t)net * nblk + b) * NE + e];
  fold[((int64_t)net * ST_LS_FOLD + sl) * NE + e] = v;
}

void launch_st_lsfold(hipStream_t st, int M1, int nets, int nblk, const double *part, double *fold) {
  const int NE = SNF * SNF + SNF * M1;
  hipLaunchKernelGGL(k_st_lsfold, dim3((NE + 255) / 256, nets, ST_LS_FOLD), dim3(256), 0, st, NE, nblk, part, fold);
}

// ---------------------------------------------------------------------------
// 4b. reduce the partials, Cholesky of A + lambda I, solve for every output
//     column; optional 16-bit rounding of W3 and the b3 correction
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_st_solve(StSolveArgs a) {
  extern __shared__ double vsh[];
  const int M1 = a.M1;
  const int NE = SNF * SNF + SNF * M1;
  const int net = blockIdx.x, tid = threadIdx.x;
  double *A = vsh;               // [SNF][SNF] (normal matrix, kept)
  double *Lc = A + SNF * SNF;    // [SNF][SNF] Cholesky factor
  double *B = Lc + SNF * SNF;    // [SNF][M1]
  __shared__ int bad;
  const double *pn = a.part + (int64_t)net * a.nblk * NE;
  for (int e = tid; e < NE; e += blockDim.x) {
    // the partials in order, eight loads in flight before their adds
    double v = 0.0;
    int b = 0;
    for (; b + 8 <= a.nblk; b += 8) {
      double x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = pn[(int64_t)(b + k) * NE + e];
#pragma unroll
      for (int k = 0; k < 8; ++k) v += x[k];
    }
    for (; b < a.nblk; ++b) v += pn[(int64_t)b * NE + e];
    if (e < SNF * SNF) A[e] = v;
    else B[e - SNF * SNF] = v;
  }
  __syncthreads();
  __shared__ double lam;
  if (tid == 0) {
    bad = A[SNF * SNF - 1] > 0.0 ? 0 : 2;
    double tr = 0.0;
    for (int i = 0; i < SNF; ++i) tr += A[i * SNF + i];
    lam = a.ridge * tr / SNF;
  }
  __syncthreads();
  for (int e = tid; e < SNF * SNF; e += blockDim.x) Lc[e] = A[e] + ((e % (SNF + 1)) == 0 ? lam : 0.0);
  __syncthreads();
  // Cholesky, column by column: the diagonal on one thread, the rows below
  // it in parallel (each entry's arithmetic as in the sequential order)
  for (int j = 0; j < SNF; ++j) {
    if (tid == 0 && bad == 0) {
      double dgn = Lc[j * SNF + j];
      for (int k = 0; k < j; ++k) dgn -= Lc[j * SNF + k] * Lc[j * SNF + k];
      if (dgn > 0.0) Lc[j * SNF + j] = sqrt(dgn);
      else bad = 1;
    }
    __syncthreads();
    if (bad) break;
    const double ljj = Lc[j * SNF + j];
    for (int i = j + 1 + tid; i < SNF; i += blockDim.x) {
      double v = Lc[i * SNF + j];
      for (int k = 0; k < j; ++k) v -= Lc[i * SNF + k] * Lc[j * SNF + k];
      Lc[i * SNF + j] = v / ljj;
    }
    __syncthreads();
  }
  if (tid == 0) a.status[net] = bad;
  if (bad) return;
  for (int o = tid; o < M1; o += blockDim.x) {
    double y[SNF];
    for (int i = 0; i < SNF; ++i) {
      double v = B[i * M1 + o];
      for (int k = 0; k < i; ++k) v -= Lc[i * SNF + k] * y[k];
      y[i] = v / Lc[i * SNF + i];
    }
    for (int i = SNF - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < SNF; ++k) v -= Lc[k * SNF + i] * y[k];
      y[i] = v / Lc[i * SNF + i];
    }
    // W3 as the kernels will hold it, then b3 = mean residual given W3
    double r = B[(SNF - 1) * M1 + o];
    for (int k = 0; k < SH2; ++k) {
      y[k] = st_round16((float)y[k], a.quant);
      r -= A[(SNF - 1) * SNF + k] * y[k];
    }
    y[SH2] = r / A[SNF * SNF - 1];
    for (int i = 0; i < SNF; ++i) a.X[((int64_t)net * SNF + i) * M1 + o] = y[i];
  }
}

void launch_st_solve(hipStream_t st, const StSolveArgs &a) {
  const size_t shm = sizeof(double) * ((size_t)2 * SNF * SNF + (size_t)SNF * a.M1);
  hipLaunchKernelGGL(k_st_solve, dim3(a.nets), dim3(256), shm, st, a);
}

// ---------------------------------------------------------------------------
// held-out check of the fitted student in FP64: sum of squared error and of
// squared teacher output per block of 64 samples
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_st_check(StCheckArgs a) {
  const int M1 = a.M1;
  const StudentLayout L = student_layout(M1);
  const int net = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  __shared__ double red[2][64];
  const int64_t q = (int64_t)net * a.batch + (int64_t)blk * 64 + tid;
  const double w = (double)a.wt[q];
  const float *P = a.params + (int64_t)net * L.np;
  const double *X = a.X + (int64_t)net * SNF * M1;
  double h2[SH2];
  st_hidden_f64(P, L, a.quant, a.s[q], h2);
  double e2 = 0.0, g2 = 0.0;
  const double *Gt = a.G + q * M1;
  for (int o = 0; o < M1; ++o) {
    double g = X[SH2 * M1 + o];
#pragma unroll
    for (int k = 0; k < SH2; ++k) g += h2[k] * X[k * M1 + o];
    const double d = g - Gt[o];
    e2 += w * d * d;
    g2 += w * Gt[o] * Gt[o];
  }
  red[0][tid] = e2;
  red[1][tid] = g2;
  __syncthreads();
  if (tid < 2) {
    double v = 0.0;
    for (int m = 0; m < 64; ++m) v += red[tid][m];
    a.part[((int64_t)net * gridDim.x + blk) * 2 + tid] = v;
  }
}

void launch_st_check(hipStream_t st, const StCheckArgs &a) {
  hipLaunchKernelGGL(k_st_check, dim3(a.batch / 64, a.nets), dim3(64), 0, st, a);
}

// ---------------------------------------------------------------------------
// force RMSE between two force arrays (the judge): fixed-order two-stage sum
// ---------------------------------------------------------------------------
constexpr int FR_BLOCKS = 256;

__global__ void k_frmse1(const double *fa, const double *fb, int64_t n, double *part) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = fa[i] - fb[i];
    v += d * d;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_frmse2(const double *part, int np, int64_t n, double *out) {
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int b = 0; b < np; ++b) v += part[b];
    out[0] = n > 0 ? sqrt(v / (double)n) : 0.0;
  }
}

void launch_force_rmse(hipStream_t st, const double *fa, const double *fb, int64_t n, double *part, double *out) {
  hipLaunchKernelGGL(k_frmse1, dim3(FR_BLOCKS), dim3(256), 0, st, fa, fb, n, part);
  hipLaunchKernelGGL(k_frmse2, dim3(1), dim3(64), 0, st, part, FR_BLOCKS, n, out);
}

// ---------------------------------------------------------------------------
// sampled judge: atoms of a cube, and the cube grown by rc (whose energies
// the cube's forces depend on)
// ---------------------------------------------------------------------------
__device__ inline double judge_min_image(double v, double L) {
  if (v > 0.5 * L) v -= L;
  else if (v < -0.5 * L) v += L;
  return v;
}

__global__ void k_judge_mark(int64_t n, const double4 *__restrict__ xw, double c0, double c1, double c2, double L0,
                             double L1, double L2, double h, double hr, int32_t *mark) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 p = xw[i];
  const double dx = fabs(judge_min_image(p.x - c0, L0)), dy = fabs(judge_min_image(p.y - c1, L1)),
               dz = fabs(judge_min_image(p.z - c2, L2));
  const double m = fmax(dx, fmax(dy, dz));
  mark[i] = m <= h ? 2 : (m <= hr ? 1 : 0);
}

void launch_judge_mark(hipStream_t st, int64_t n, const double4 *xw, const double *c, const double *L, double h,
                       double hr, int32_t *mark) {
  if (n > 0)
    hipLaunchKernelGGL(k_judge_mark, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, xw, c[0], c[1], c[2],
                       L[0], L[1], L[2], h, hr, mark);
}

// force RMSE over the atoms with mark == 2: part[2 b] = sum |dF|^2, part[2 b + 1] = count
__global__ void k_frmse1m(const double *fa, const double *fb, int64_t n, const int32_t *mark, double *part) {
  __shared__ double red[2][256];
  double v = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (mark[i] != 2) continue;
    const double dx = fa[3 * i] - fb[3 * i], dy = fa[3 * i + 1] - fb[3 * i + 1], dz = fa[3 * i + 2] - fb[3 * i + 2];
    v += dx * dx + dy * dy + dz * dz;
    c += 1.0;
  }
  red[0][threadIdx.x] = v;
  red[1][threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_frmse2m(const double *part, int np, double *out, double *count) {
  if (threadIdx.x == 0) {
    double v = 0.0, c = 0.0;
    for (int b = 0; b < np; ++b) {
      v += part[2 * b];
      c += part[2 * b + 1];
    }
    out[0] = c > 0 ? sqrt(v / c) : 0.0;
    count[0] = c;
  }
}

void launch_force_rmse_masked(hipStream_t st, const double *fa, const double *fb, int64_t n, const int32_t *mark,
                              double *part, double *out, double *count) {
  hipLaunchKernelGGL(k_frmse1m, dim3(FR_BLOCKS), dim3(256), 0, st, fa, fb, n, mark, part);
  hipLaunchKernelGGL(k_frmse2m, dim3(1), dim3(64), 0, st, part, FR_BLOCKS, out, count);
}

__global__ void k_copy_i32(const int32_t *src, int32_t *dst) {
  if (threadIdx.x == 0) *dst = *src;
}

void launch_copy_i32(hipStream_t st, const int32_t *src, int32_t *dst) {
  hipLaunchKernelGGL(k_copy_i32, dim3(1), dim3(64), 0, st, src, dst);
}

}  // namespace dpk
