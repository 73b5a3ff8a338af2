// Double-precision embedding net + descriptor (and the same kernels in
// single precision for DP_MIX_FP32, the paper's MIX-32 scheme, Section V-B
// "Mixed-precision computation"), fused per centre atom so the
// embedding matrix G never reaches HBM (Section V-B, "Increasing
// computational granularity": the type-sorted, padded list lets every tile
// of neighbours use one net without branching).
//
// Pass 1 (forward):  for each real neighbour j of atom i (net (t_i, t_j)),
//   G_j = Emb(s_j)  (1 -> w1 on VALU, later layers on MFMA),
//   T  += G_j R_j^T            (MFMA, K = neighbours)
//   T  *= 1/Nc,  D = T T_<^T   (MFMA, K = 4)
// Pass 2 (backward): dT = (dD T_< + [a < M2] dD^T T) / Nc, then per tile the
//   net is re-run in forward tangent mode (h and dh/ds side by side, the
//   second MFMA column tile), giving G_j and G'_j = dG_j/ds_j in registers:
//   dE/dR_j = G_j^T dT,   dE/ds_j += (dT R_j) . G'_j,
//   g_ij = sum_k dE/dR_jk dR_jk/dr_ij,  F_i += g_ij, F_j -= g_ij (atomics),
//   Xi -= g_ij (x) r_ij (per-block partial sums, reduced in block order).
// This fuses the paper's ProdForce and ProdVirial operators into the
// embedding backward.
//
// Matrix layout.  For v_mfma_f64_16x16x4: A lane l holds A[l%16][l/16],
// B lane l holds B[l/16][l%16], and D register r of lane l is
// D[4r + l/16][l%16] (the f64 variant interleaves rows by register, unlike
// the f32-output variants).  The backward computes each layer transposed,
// Z^T[out x 16] = W^T H^T, with the 16 neighbours of a tile as the N
// dimension and activations in a per-wave LDS tile [feature][neighbour].
// The forward swaps the operands of the same loads, Z[16 x out] = H W with
// the neighbours as M, so that the last layer's output registers are
// directly the B operand of T^T += R^T G; its LDS tiles are
// [neighbour][feature] with an odd row stride.  Weights stream from L2 in
// their padded [K][M] layout; layer 0's weights are copied to LDS per net.
#include "dp_f64.h"

namespace dpk {

constexpr int EMB_WAVES = 2;

struct EmbLds {
  int rows[2];  // rows of the two ping-pong activation buffers
  int cols;     // 16 (forward) or 32 (tangent pass)
  int ld[2];    // forward: row stride of the [16 neighbours][features] buffers
  int v0;       // backward of a three-layer net: buffer 0 holds layer 0's values only (16 columns)
  int off_buf[2], off_rt, off_t, off_g, per_wave;  // offsets in doubles
};

// per-wave LDS (doubles): the ping-pong activation buffers of the hidden
// layers (the last layer's output is not stored), the tile's R rows [16][4]
// and T (forward: the unscaled sum; backward: dT) [M1 padded][4]. The
// forward's buffers are [16 neighbours][ld] with an odd stride ld, so that
// both a feature column (the MFMA A operand) and a neighbour row (the
// epilogue's stores) spread over the banks; the backward's are
// [feature][cols] (value and tangent side by side).
static EmbLds emb_lds_layout(const Dims &d, int pass, bool values_only) {
  EmbLds L{};
  L.cols = pass == 1 ? 16 : 32;
  for (int l = 0; l < d.n_emb - 1; ++l) {
    const int r = d.ekp[l + 1];
    if (r > L.rows[l & 1]) L.rows[l & 1] = r;
  }
  if (pass == 1) {
    L.ld[0] = L.rows[0] | 1;
    L.ld[1] = L.rows[1] | 1;
    L.off_buf[0] = 0;
    L.off_buf[1] = 16 * L.ld[0];
    L.off_rt = L.off_buf[1] + 16 * L.ld[1];
    L.off_t = L.off_rt + 64;
    L.off_g = L.off_t + d.emp[d.n_emb] * 4;
    L.per_wave = L.off_g + 2 * d.ekp[1];  // + layer 0's weights and biases
    return L;
  }
  // backward of a three-layer net whose first layer has no skip: layer 0's
  // tangents are recomputed from its values as layer 1 reads them, and the
  // tile's s values come by lane shuffles, so buffer 0 holds 16 columns and
  // there is no R tile -- with dT unpadded, the wave's area fits four
  // two-wave workgroups per CU in FP64. The FP32 twin is bound by registers,
  // not LDS, and keeps the stored tangents (the recompute only costs it).
  L.v0 = (values_only && pass == 2 && d.n_emb == 3 && d.ew[1] > 2) ? 1 : 0;
  const int c0 = L.v0 ? 16 : L.cols;
  if (pass == 2) {
    // the backward stages an atom's dD row and T in the two buffers first
    const int need = d.M1 * d.M2 + 4 * d.M1, have = L.rows[0] * c0 + L.rows[1] * L.cols;
    if (need > have) L.rows[1] += (need - have + L.cols - 1) / L.cols;
  }
  L.off_buf[0] = 0;
  L.off_buf[1] = L.rows[0] * c0;
  L.off_rt = L.off_buf[1] + L.rows[1] * L.cols;
  L.off_t = L.off_rt + (L.v0 ? 0 : 64);
  L.off_g = L.off_t + (L.v0 ? d.M1 : d.emp[d.n_emb]) * 4;
  // FP64 backward: layer 0's weights, zero past its width, at off_g (read
  // by the values-only layer-1 operand loader)
  L.per_wave = L.off_g + (values_only && pass == 2 ? d.ekp[1] : 0);
  return L;
}


// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
template <typename Real>
__global__ void __launch_bounds__(64 * EMB_WAVES) k_embed_fwd_f64(EmbedArgsT<Real, typename MF<Real>::vec4> a,
                                                                EmbLds L) {
  extern __shared__ __align__(16) unsigned char emb_smem[];
  Real *smem = (Real *)emb_smem;
  const Dims &d = a.d;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  Real *lds = smem + wv * L.per_wave;
  Real *Rl = lds + L.off_rt;
  Real *Tl = lds + L.off_t;
  Real *W0s = lds + L.off_g, *b0s = W0s + d.ekp[1];
  const int64_t nwaves = (int64_t)gridDim.x * EMB_WAVES;
  const int64_t gw = (int64_t)blockIdx.x * EMB_WAVES + wv;
  const int64_t chunk = (a.rows + nwaves - 1) / nwaves;
  const int64_t p_end = (gw + 1) * chunk < a.rows ? (gw + 1) * chunk : a.rows;
  const int nmtG = d.emp[d.n_emb] >> 4;
  const int M1p = d.emp[d.n_emb];
  const int MM = d.M1 * d.M2;

  for (int64_t p = gw * chunk; p < p_end; ++p) {
    const int i = a.atom_of_pos[p];
    Real *Dp = a.D + p * (int64_t)MM;
    if (i < 0) {
      for (int o = lane; o < MM; o += 64) Dp[o] = 0.0;
      continue;
    }
    const int t = (int)a.xw[i].w;
    // T accumulates in LDS (unscaled): lane (g, c) owns T[f][c] for its rows f
    for (int o = lane; o < M1p * 4; o += 64) Tl[o] = 0.0;

    for (int u = 0; u < d.ntypes; ++u) {
      const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
      const int64_t base = (int64_t)i * d.nnei + d.off[u];
      if (cnt == 0) continue;
      // layer 0's weights and biases in LDS, zero past its width, so that
      // the layer-0 loop has no branch around global loads (read after the
      // barrier that follows the R rows)
      {
        const Real *W0 = a.ew + a.eo.w[t][u][0];
        const Real *b0 = a.ew + a.eo.b[t][u][0];
        for (int o = lane; o < d.ekp[1]; o += 64) {
          W0s[o] = o < d.ew[1] ? W0[o] : Real(0);
          b0s[o] = o < d.ew[1] ? b0[o] : Real(0);
        }
      }
      // environment rows one tile ahead (unconditional loads: slots past the
      // block reread its last row and are zeroed when used)
      typename MF<Real>::vec4 r4n = a.rt[base + (lane < cnt ? lane : cnt - 1)];
      for (int n0 = 0; n0 < cnt; n0 += 16) {
        typename MF<Real>::vec4 r4 = r4n;
        r4n = a.rt[base + (n0 + 16 + lane < cnt ? n0 + 16 + lane : cnt - 1)];
        if (lane < 16) {
          if (n0 + lane >= cnt) r4 = MF<Real>::zero4();
          Rl[lane * 4 + 0] = r4.x;
          Rl[lane * 4 + 1] = r4.y;
          Rl[lane * 4 + 2] = r4.z;
          Rl[lane * 4 + 3] = r4.w;
        }
        wave_sync();
        // layer 0: 1 -> ew[1] on VALU
        {
          const int out1 = d.ew[1];
          const int rows = d.ekp[1];
          Real *H = lds + L.off_buf[0];
          for (int idx = lane; idx < rows * 16; idx += 64) {
            const int f = idx >> 4, n = idx & 15;
            const Real s = Rl[n * 4];
            // padded features: tanh(0) = 0
            Real h = MF<Real>::tanh_(s * W0s[f] + b0s[f]);
            if (out1 == 1 || out1 == 2) h += f < out1 ? s : Real(0);
            H[n * L.ld[0] + f] = h;
          }
        }
        wave_sync();
        // layers 1 .. n_emb-1 on MFMA, EMB_G output tiles at a time, with
        // the tile's neighbours as the M dimension: Z[n][f] = sum_k H[n][k]
        // W[k][f], so register r of lane (g, c) holds neighbour row(r, g) of
        // feature 16 mt + c. The last layer's registers are then directly the
        // B operand of T^T[c'][f] += sum_n R[n][c'] G[n][f] (k-step r takes
        // register r; A holds R at the same neighbours), and G never goes to
        // LDS.
        // A operands of that product for this tile: R[row(kn, g)][c'] for
        // c' = lane % 16 < 4, zero for the 12 unused output rows
        Real ra[4];
#pragma unroll
        for (int kn = 0; kn < 4; ++kn)
          ra[kn] = (lane & 15) < 4 ? Rl[MF<Real>::row(kn, lane >> 4) * 4 + (lane & 15)] : Real(0);
        for (int l = 1; l < d.n_emb; ++l) {
          const int in = d.ew[l], out = d.ew[l + 1];
          const bool last = l == d.n_emb - 1;
          const Real *Hin = lds + L.off_buf[(l - 1) & 1];
          Real *Hout = lds + L.off_buf[l & 1];
          const int ldi = L.ld[(l - 1) & 1], ldo = L.ld[l & 1];
          const int rows_out = last ? 0 : d.ekp[l + 1];
          const Real *W = a.ew + a.eo.w[t][u][l];
          const Real *bias = a.ew + a.eo.b[t][u][l];
          const int nmt = d.emp[l + 1] >> 4;
          // A operand of k-step kk: H[n = lane % 16][kk + lane / 16]
          const Real *hr = Hin + (lane & 15) * ldi + (lane >> 4);
          for (int mt0 = 0; mt0 < nmt; mt0 += EMB_G) {
            typename MF<Real>::acc acc[1][EMB_G];
            mfma_group_b<1, true>(
                W, d.ekp[l], d.emp[l + 1], [&](int kk, int) { return hr[kk]; }, lane, mt0, acc);
#pragma unroll
            for (int g = 0; g < EMB_G; ++g) {
              const int mt = mt0 + g;
              if (mt < nmt) {
                const int f = mt * 16 + (lane & 15);
                Real hreg[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int n = MF<Real>::row(r, lane >> 4);
                  Real h = 0;
                  if (f < out) {
                    const Real z = acc[0][g][r] + bias[f];
                    h = (d.emb_lin && last) ? z : MF<Real>::tanh_(z);
                    const int sf = skip_src(f, in, out);
                    if (sf >= 0) h += Hin[n * ldi + sf];
                  }
                  hreg[r] = h;
                  if (!last && f < rows_out) Hout[n * ldo + f] = h;
                }
                if (last) {
                  // register r of lane (g', c) holds T^T[row(r, g')][16 mt + c];
                  // rows below 4 are T's components, each owned by one lane
                  typename MF<Real>::acc tacc;
#pragma unroll
                  for (int r = 0; r < 4; ++r) {
                    const int c = MF<Real>::row(r, lane >> 4);
                    tacc[r] = c < 4 ? Tl[f * 4 + c] : Real(0);
                  }
#pragma unroll
                  for (int kn = 0; kn < 4; ++kn) tacc = MF<Real>::mma(ra[kn], hreg[kn], tacc);
#pragma unroll
                  for (int r = 0; r < 4; ++r) {
                    const int c = MF<Real>::row(r, lane >> 4);
                    if (c < 4) Tl[f * 4 + c] = tacc[r];
                  }
                }
              }
            }
          }
          wave_sync();
        }
      }
    }
    // T = sum / Nc -> global and LDS
    {
      Real *Tg = a.T + (int64_t)i * d.M1 * 4;
      for (int o = lane; o < M1p * 4; o += 64) {
        const Real v = Tl[o] * (Real)d.inv_nc;
        Tl[o] = v;
        if ((o >> 2) < d.M1) Tg[o] = v;
      }
    }
    wave_sync();
    // D = T T_<^T : one MFMA step of K = 4 per output tile
    {
      const int b = lane & 15;
      const Real bv = b < d.M2 ? Tl[b * 4 + (lane >> 4)] : Real(0);
      for (int mt = 0; mt < nmtG; ++mt) {
        typename MF<Real>::acc z = MF<Real>::mma(Tl[(mt * 16 + (lane & 15)) * 4 + (lane >> 4)], bv,
                                                 typename MF<Real>::acc{0, 0, 0, 0});
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int f = mt * 16 + MF<Real>::row(r, lane >> 4);
          if (f < d.M1 && b < d.M2) Dp[f * d.M2 + b] = z[r];
        }
      }
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
__device__ inline void switch_fn(double r, double rcs, double rc, double inv_w, double &sw, double &dsw) {
  if (r < rcs) {
    sw = 1.0;
    dsw = 0.0;
  } else if (r < rc) {
    const double x = (r - rcs) * inv_w;
    sw = x * x * x * (-6.0 * x * x + 15.0 * x - 10.0) + 1.0;
    dsw = x * x * (-30.0 * x * x + 60.0 * x - 30.0) * inv_w;
  } else {
    sw = 0.0;
    dsw = 0.0;
  }
}

template <typename Real>
__global__ void __launch_bounds__(64 * EMB_WAVES) __attribute__((amdgpu_waves_per_eu(2)))
k_embed_bwd_f64(EmbedArgsT<Real, typename MF<Real>::vec4> a, EmbLds L) {
  extern __shared__ __align__(16) unsigned char emb_smem[];
  Real *smem = (Real *)emb_smem;
  __shared__ double vred[EMB_WAVES][9];
  const Dims &d = a.d;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  Real *lds = smem + wv * L.per_wave;
  Real *Rl = lds + L.off_rt;
  Real *dTl = lds + L.off_t;
  Real *W0l = lds + L.off_g;
  // the values-only layer-0 layout exists for FP64 only: the FP32 build folds
  // it away and keeps the stored-tangent code as it was
  const bool v0 = sizeof(Real) == sizeof(double) && L.v0;
  const int64_t nwaves = (int64_t)gridDim.x * EMB_WAVES;
  const int64_t gw = (int64_t)blockIdx.x * EMB_WAVES + wv;
  const int64_t chunk = (a.rows + nwaves - 1) / nwaves;
  const int64_t p_end = (gw + 1) * chunk < a.rows ? (gw + 1) * chunk : a.rows;
  const int MM = d.M1 * d.M2;
  const int M1p = d.emp[d.n_emb];
  const double rc = d.rcut, rcs = d.rcut_smth, inv_w = 1.0 / (d.rcut - d.rcut_smth);
  double vir[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = 0.0;

  for (int64_t p = gw * chunk; p < p_end; ++p) {
    const int i = a.atom_of_pos[p];
    if (i < 0) continue;
    const int t = (int)a.xw[i].w;
    // dT / Nc, from the atom's dD row and T staged in the activation buffers
    // (free until the first tile): one coalesced pass of loads, all in
    // flight together, then the sums from LDS in the same order as before
    {
      Real *dDs = lds + L.off_buf[0];
      Real *Ts = dDs + MM;
      const Real *Ti = a.T + (int64_t)i * d.M1 * 4;
      const Real *dDp = a.dD + p * (int64_t)MM;
      for (int o = lane; o < MM; o += 64) dDs[o] = dDp[o];
      for (int o = lane; o < d.M1 * 4; o += 64) Ts[o] = Ti[o];
      wave_sync();
      for (int o = lane; o < (v0 ? d.M1 : M1p) * 4; o += 64) {
        const int f = o >> 2, k = o & 3;
        Real v = 0;
        if (f < d.M1) {
          for (int b = 0; b < d.M2; ++b) v += dDs[f * d.M2 + b] * Ts[b * 4 + k];
          if (f < d.M2)
            for (int a2 = 0; a2 < d.M1; ++a2) v += dDs[a2 * d.M2 + f] * Ts[a2 * 4 + k];
        }
        dTl[o] = v * (Real)d.inv_nc;
      }
    }
    wave_sync();
    double fi0 = 0.0, fi1 = 0.0, fi2 = 0.0;
    for (int u = 0; u < d.ntypes; ++u) {
      const int cnt = a.nreal[(int64_t)i * d.ntypes + u];
      const int64_t base = (int64_t)i * d.nnei + d.off[u];
      const Real *W0 = a.ew + a.eo.w[t][u][0];
      const Real *b0 = a.ew + a.eo.b[t][u][0];
      // layer 0's weights for the formed tangents, from LDS: a global load
      // there sat in a branch that waited for every load in flight (read
      // after the barrier that follows layer 0)
      if (v0)
        for (int o = lane; o < d.ekp[1]; o += 64) W0l[o] = o < d.ew[1] ? W0[o] : Real(0);
      for (int n0 = 0; n0 < cnt; n0 += 16) {
        const bool valid = lane < 16 && n0 + lane < cnt;
        typename MF<Real>::vec4 R4 = MF<Real>::zero4();
        double4 D4 = make_double4(0.0, 0.0, 0.0, 1.0);
        int j = -1;
        if (valid) {
          R4 = a.rt[base + n0 + lane];
          D4 = a.dr[base + n0 + lane];
          j = a.nlist[base + n0 + lane];
        }
        // the tile's s values: neighbour n = lane % 16 of every lane (lanes
        // n < 16 hold their rows); through LDS unless the layout has no R tile
        Real s_n;
        if (v0) {
          s_n = __shfl(R4.x, lane & 15);
        } else {
          if (lane < 16) {
            Rl[lane * 4 + 0] = R4.x;
            Rl[lane * 4 + 1] = R4.y;
            Rl[lane * 4 + 2] = R4.z;
            Rl[lane * 4 + 3] = R4.w;
          }
          wave_sync();
          s_n = Rl[(lane & 15) * 4];
        }
        // layer 0 with tangent: h and dh/ds side by side (columns 0..15,
        // 16..31), or h alone (v0)
        const int out1 = d.ew[1];
        {
          Real *H = lds + L.off_buf[0];
          for (int idx = lane; idx < d.ekp[1] * 16; idx += 64) {
            const int f = idx >> 4, n = idx & 15;
            const Real s = s_n;
            Real h = 0, hd = 0;
            if (f < out1) {
              const Real th = MF<Real>::tanh_(s * W0[f] + b0[f]);
              h = th;
              hd = (Real(1) - th * th) * W0[f];
              if (out1 == 1 || out1 == 2) {
                h += s;
                hd += Real(1);
              }
            }
            if (v0) {
              H[f * 16 + n] = h;
            } else {
              H[f * 32 + n] = h;
              H[f * 32 + 16 + n] = hd;
            }
          }
        }
        wave_sync();
        Real ga[4] = {0, 0, 0, 0}, gb[4] = {0, 0, 0, 0};
        for (int l = 1; l < d.n_emb; ++l) {
          const int in = d.ew[l], out = d.ew[l + 1];
          const bool last = (l == d.n_emb - 1);
          const Real *Hin = lds + L.off_buf[(l - 1) & 1];
          Real *Hout = lds + L.off_buf[l & 1];
          const int rows_out = last ? 0 : d.ekp[l + 1];
          const Real *W = a.ew + a.eo.w[t][u][l];
          const Real *bias = a.ew + a.eo.b[t][u][l];
          const int nmt = d.emp[l + 1] >> 4;
          // layer 0's values only (v0): its tangent (1 - h^2) w0 is formed
          // here, the same expression the layer-0 loop evaluates
          const bool hv = v0 && l == 1;
          const int cin = hv ? 16 : 32;
          const Real *hr = Hin + (lane >> 4) * cin + (lane & 15);
          for (int mt0 = 0; mt0 < nmt; mt0 += EMB_G) {
            typename MF<Real>::acc acc[2][EMB_G];
            // one instantiation for both layouts: the tangent column reads
            // the stored tangent or forms it (the other operand is selected
            // away; the loads stay inside the buffers)
            mfma_group_b<2>(
                W, d.ekp[l], d.emp[l + 1],
                [&](int kk, int ct) {
                  const Real h = hr[kk * cin];
                  if (ct == 0) return h;
                  const Real formed = (Real(1) - h * h) * W0l[kk + (lane >> 4)];
                  return hv ? formed : hr[kk * cin + (hv ? 0 : 16)];
                },
                lane, mt0, acc);
#pragma unroll
            for (int g = 0; g < EMB_G; ++g) {
              const int mt = mt0 + g;
              if (mt >= nmt) continue;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int f = mt * 16 + MF<Real>::row(r, lane >> 4), n = lane & 15;
                Real h = 0, hd = 0;
                if (f < out) {
                  const Real z = acc[0][g][r] + bias[f];
                  const bool lin = d.emb_lin && last;
                  const Real th = lin ? z : MF<Real>::tanh_(z);
                  h = th;
                  hd = lin ? acc[1][g][r] : (Real(1) - th * th) * acc[1][g][r];
                  const int sf = skip_src(f, in, out);
                  if (sf >= 0) {
                    const Real hs = Hin[sf * cin + n];
                    h += hs;
                    hd += hv ? (Real(1) - hs * hs) * W0l[sf] : Hin[sf * 32 + 16 + n];
                  }
                }
                if (last) {
                  if (f < out) {
                    const Real *dt = dTl + f * 4;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                      ga[k] += h * dt[k];
                      gb[k] += hd * dt[k];
                    }
                  }
                } else if (f < rows_out) {
                  Hout[f * 32 + n] = h;
                  Hout[f * 32 + 16 + n] = hd;
                }
              }
            }
          }
          wave_sync();
        }
        // sum the four lane groups: lanes n, n+16, n+32, n+48 share neighbour n
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          ga[k] += __shfl_xor(ga[k], 16);
          ga[k] += __shfl_xor(ga[k], 32);
          gb[k] += __shfl_xor(gb[k], 16);
          gb[k] += __shfl_xor(gb[k], 32);
        }
        if (valid) {
          // dE/dR_j (the 1/Nc is inside dT; in the network's precision); the
          // embedding path adds to the s component; the Jacobian in FP64
          const double g0 = (double)(ga[0] + (R4.x * gb[0] + R4.y * gb[1] + R4.z * gb[2] + R4.w * gb[3]));
          const double g1 = (double)ga[1], g2 = (double)ga[2], g3 = (double)ga[3];
          if (a.net_deriv) {
            double *nd = a.net_deriv + (base + n0 + lane) * 4;
            nd[0] = g0;
            nd[1] = g1;
            nd[2] = g2;
            nd[3] = g3;
          }
          const double dx = D4.x, dy = D4.y, dz = D4.z, r = D4.w;
          double sw, dsw;
          switch_fn(r, rcs, rc, inv_w, sw, dsw);
          const double ir = 1.0 / r;
          const double s = sw * ir;
          const double ds = (dsw * r - sw) * ir * ir;
          const double tt = s * ir;
          const double dtt = dsw * ir * ir - 2.0 * sw * ir * ir * ir;
          const double gd = g1 * dx + g2 * dy + g3 * dz;
          const double c = (g0 * ds + dtt * gd) * ir;
          const double gx = c * dx + tt * g1, gy = c * dy + tt * g2, gz = c * dz + tt * g3;
          fi0 += gx;
          fi1 += gy;
          fi2 += gz;
          unsafeAtomicAdd(a.force + 3 * (int64_t)j + 0, -gx);
          unsafeAtomicAdd(a.force + 3 * (int64_t)j + 1, -gy);
          unsafeAtomicAdd(a.force + 3 * (int64_t)j + 2, -gz);
          vir[0] -= gx * dx; vir[1] -= gx * dy; vir[2] -= gx * dz;
          vir[3] -= gy * dx; vir[4] -= gy * dy; vir[5] -= gy * dz;
          vir[6] -= gz * dx; vir[7] -= gz * dy; vir[8] -= gz * dz;
        }
        wave_sync();
      }
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
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
    for (int w = 0; w < EMB_WAVES; ++w) v += vred[w][threadIdx.x];
    a.vir_part[(int64_t)blockIdx.x * 9 + threadIdx.x] = v;
  }
}

static int emb_grid(int64_t rows) {
  int64_t g = (rows + EMB_WAVES - 1) / EMB_WAVES;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

int embed_bwd_grid(int64_t rows) { return emb_grid(rows); }

template <typename Real>
static void launch_fwd_t(hipStream_t s, const EmbedArgsT<Real, typename MF<Real>::vec4> &a) {
  EmbLds L = emb_lds_layout(a.d, 1, false);
  size_t shm = sizeof(Real) * (size_t)L.per_wave * EMB_WAVES;
  hipLaunchKernelGGL(k_embed_fwd_f64<Real>, dim3(emb_grid(a.rows)), dim3(64 * EMB_WAVES), shm, s, a, L);
}

template <typename Real>
static void launch_bwd_t(hipStream_t s, const EmbedArgsT<Real, typename MF<Real>::vec4> &a, int grid) {
  EmbLds L = emb_lds_layout(a.d, 2, sizeof(Real) == sizeof(double));
  size_t shm = sizeof(Real) * (size_t)L.per_wave * EMB_WAVES;
  hipLaunchKernelGGL(k_embed_bwd_f64<Real>, dim3(grid), dim3(64 * EMB_WAVES), shm, s, a, L);
}

void launch_embed_fwd_f64(hipStream_t s, const EmbedArgs &a) { launch_fwd_t<double>(s, a); }
void launch_embed_bwd_f64(hipStream_t s, const EmbedArgs &a, int grid) { launch_bwd_t<double>(s, a, grid); }
void launch_embed_fwd_f32(hipStream_t s, const EmbedArgs32 &a) { launch_fwd_t<float>(s, a); }
void launch_embed_bwd_f32(hipStream_t s, const EmbedArgs32 &a, int grid) { launch_bwd_t<float>(s, a, grid); }

// LDS bytes of the larger of the FP64 kernels' two layouts; the FP32
// kernels take half of the stored-tangent one
size_t embed_lds_bytes(const Dims &d, int pass) {
  EmbLds L = emb_lds_layout(d, pass, false), V = emb_lds_layout(d, pass, true);
  return sizeof(double) * (size_t)(L.per_wave > V.per_wave ? L.per_wave : V.per_wave) * EMB_WAVES;
}

}  // namespace dpk
