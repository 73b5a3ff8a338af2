// Host runtime of the C ABI declared in include/dpmi.h: model-blob parsing,
// device weight layout, the workspace arena (allocated once, grown only when
// a larger system arrives -- the paper's "trunk of GPU memory", Section
// V-A), and the launch sequence of one evaluation and of the MD loop.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dp_internal.h"
#include "dp_mix.h"
#include "dpmi.h"

using namespace dpk;

namespace dpk {
size_t embed_lds_bytes(const Dims &d, int pass);
}

namespace {

constexpr double MVV2E = 103.642696562;
constexpr double KB_EV = 8.617333262e-5;

// ---------------------------------------------------------------------------
// model blob
// ---------------------------------------------------------------------------
struct HostModel {
  int64_t ntypes = 0, n_emb = 0, n_fit = 0, M2 = 0;
  double rcut = 0, rcut_smth = 0, desc_norm = 1;
  std::vector<int64_t> sel, emb_w, fit_w;  // emb_w[0..n_emb], fit_w[0..n_fit+1]
  std::vector<std::vector<double>> eW, eb, fW, fb;
  size_t eidx(int64_t t, int64_t u, int64_t l) const { return (size_t)((t * ntypes + u) * n_emb + l); }
  size_t fidx(int64_t t, int64_t l) const { return (size_t)(t * (n_fit + 1) + l); }
};

class Reader {
 public:
  Reader(const unsigned char *p, size_t n) : p_(p), end_(p + n) {}
  bool i64(int64_t &v) { return take(&v, 8); }
  bool f64(double &v) { return take(&v, 8); }
  bool f64s(std::vector<double> &v, size_t n) {
    v.resize(n);
    return n == 0 || take(v.data(), 8 * n);
  }
  bool bytes(void *dst, size_t n) { return take(dst, n); }
  size_t left() const { return (size_t)(end_ - p_); }

 private:
  bool take(void *dst, size_t n) {
    if ((size_t)(end_ - p_) < n) return false;
    std::memcpy(dst, p_, n);
    p_ += n;
    return true;
  }
  const unsigned char *p_, *end_;
};

bool parse_blob(const void *blob, size_t nbytes, HostModel &m, std::string &err) {
  Reader r((const unsigned char *)blob, nbytes);
  char magic[8];
  int64_t version = 0;
  if (!r.bytes(magic, 8) || std::memcmp(magic, "DPMIBLOB", 8) != 0) return err = "blob: bad magic", false;
  if (!r.i64(version) || version != 1) return err = "blob: unsupported version", false;
  if (!r.i64(m.ntypes) || !r.i64(m.n_emb) || !r.i64(m.n_fit) || !r.i64(m.M2)) return err = "blob: truncated header", false;
  if (m.ntypes < 1 || m.ntypes > MAXT) return err = "blob: ntypes must be 1..8", false;
  if (m.n_emb < 2 || m.n_emb > MAXL) return err = "blob: embedding depth must be 2..4", false;
  if (m.n_fit < 1 || m.n_fit > MAXF) return err = "blob: fitting depth must be 1..4", false;
  if (!r.f64(m.rcut) || !r.f64(m.rcut_smth) || !r.f64(m.desc_norm)) return err = "blob: truncated header", false;
  m.sel.resize(m.ntypes);
  for (auto &s : m.sel)
    if (!r.i64(s) || s < 0) return err = "blob: bad sel", false;
  m.emb_w.resize(m.n_emb + 1);
  for (auto &w : m.emb_w)
    if (!r.i64(w) || w < 1) return err = "blob: bad embedding width", false;
  if (m.emb_w[0] != 1) return err = "blob: embedding input width must be 1", false;
  m.fit_w.resize(m.n_fit + 2);
  m.fit_w[0] = m.emb_w[m.n_emb] * m.M2;
  for (int64_t l = 1; l <= m.n_fit; ++l)
    if (!r.i64(m.fit_w[l]) || m.fit_w[l] < 1) return err = "blob: bad fitting width", false;
  m.fit_w[m.n_fit + 1] = 1;
  const int64_t T = m.ntypes;
  m.eW.resize(T * T * m.n_emb);
  m.eb.resize(T * T * m.n_emb);
  for (int64_t t = 0; t < T; ++t)
    for (int64_t u = 0; u < T; ++u)
      for (int64_t l = 0; l < m.n_emb; ++l)
        if (!r.f64s(m.eW[m.eidx(t, u, l)], m.emb_w[l] * m.emb_w[l + 1]) ||
            !r.f64s(m.eb[m.eidx(t, u, l)], m.emb_w[l + 1]))
          return err = "blob: truncated embedding weights", false;
  m.fW.resize(T * (m.n_fit + 1));
  m.fb.resize(T * (m.n_fit + 1));
  for (int64_t t = 0; t < T; ++t)
    for (int64_t l = 0; l <= m.n_fit; ++l)
      if (!r.f64s(m.fW[m.fidx(t, l)], m.fit_w[l] * m.fit_w[l + 1]) || !r.f64s(m.fb[m.fidx(t, l)], m.fit_w[l + 1]))
        return err = "blob: truncated fitting weights", false;
  if (r.left() != 0) return err = "blob: trailing bytes", false;
  return true;
}

int rup(int v, int m) { return (v + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct DevStatus {
  uint32_t flags;
  uint32_t pad;
  unsigned long long overflow;
  int32_t max_real[MAXT];
  unsigned long long nbuild;
};

struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
  int64_t n_cap = -1, rows_cap = 0, ncell_cap = 0;
  int cand_cap = 0;
  bool nd = false;
  double4 *xw = nullptr, *xref = nullptr, *rt = nullptr, *dr = nullptr;
  int32_t *cell_of, *cell_atoms, *cell_start, *cell_fill, *scan_tmp, *cand, *cand_n, *nlist, *nreal, *pos_of_atom,
      *atom_of_pos, *blk_counts, *type_count, *type_start;
  double *T, *D, *dD, *Y[MAXF + 1], *Tt[MAXF + 1], *G[MAXF + 1], *eatom, *partial, *vir_part, *force_tmp,
      *net_deriv, *energy, *virial, *ke;
  // mixed-precision buffers
  float *T32, *D32, *dD32, *Yf[MAXF + 1], *Ttf[MAXF + 1], *Gf[MAXF + 1];
  int prec = -1;  // precision the buffers were laid out for
  DevStatus *status;
};

}  // namespace

struct dp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool has_model = false;
  int precision = DP_FP64;
  HostModel hm;
  Dims dims{};
  EmbOffsets eo{};
  FitOffsets fo{};
  double *d_emb = nullptr, *d_fit = nullptr;
  // mixed-precision weights (16-bit MFMA operands + f32)
  unsigned char *d_mix_nets = nullptr, *d_fit_mix = nullptr;
  FitMixOffsets fmo{};
  int mix_shape = -1, n16 = 0;
  Workspace ws;
  DevStatus *h_status = nullptr;  // pinned
  dp_stats stats{};
  bool keep = false, timing = false;
  // per-evaluation event marks while timing is on: ev[k + 8*e]
  std::vector<hipEvent_t> ev;
  int64_t nev = 0;      // evaluations recorded since timing was enabled
  int64_t ev_cap = 0;   // evaluations the event ring holds
  int64_t last_n = 0;
  bool fwd_ready = false;  // dp_energy ran; dp_energy_backward may follow
  std::string err;
};

namespace {

int fail(dp_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, DP_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

void free_ws(Workspace &w) {
  if (w.base) (void)hipFree(w.base);
  w = Workspace{};
}

// Carve every buffer out of one allocation.  Sizes depend on n (atoms),
// the cell count and the candidate capacity.
int ensure_ws(dp_ctx *c, int64_t n, int64_t ncell, int cand_cap) {
  Workspace &w = c->ws;
  const Dims &d = c->dims;
  const bool need_nd = c->keep;
  const bool mixed = c->precision != DP_FP64;
  if (n <= w.n_cap && ncell <= w.ncell_cap && cand_cap <= w.cand_cap && (!need_nd || w.nd) &&
      w.prec == c->precision)
    return DP_OK;
  int64_t nn = std::max<int64_t>(n, w.n_cap > 0 ? (w.n_cap * 5) / 4 : n);
  nn = std::max<int64_t>(nn, 1);
  int64_t nc = std::max<int64_t>(ncell, w.ncell_cap);
  int cc = std::max(cand_cap, w.cand_cap);
  bool nd = need_nd || w.nd;
  free_ws(w);
  const int64_t rows = (nn + ROW_TILE - 1) / ROW_TILE * ROW_TILE + (int64_t)ROW_TILE * d.ntypes;
  const int64_t nblk = (nn + 255) / 256 + 1;
  size_t off = 0;
  std::vector<std::pair<void **, size_t>> plan;
  auto add = [&](void **p, size_t bytes) { plan.push_back({p, bytes}); };
  add((void **)&w.xw, sizeof(double4) * nn);
  add((void **)&w.xref, sizeof(double4) * nn);
  add((void **)&w.cell_of, 4 * nn);
  add((void **)&w.cell_atoms, 4 * nn);
  add((void **)&w.cell_start, 4 * (nc + 1));
  add((void **)&w.cell_fill, 4 * nc);
  add((void **)&w.scan_tmp, 4 * nc);
  add((void **)&w.cand, (size_t)4 * nn * cc);
  add((void **)&w.cand_n, 4 * nn);
  add((void **)&w.nlist, (size_t)4 * nn * d.nnei);
  add((void **)&w.nreal, (size_t)4 * nn * d.ntypes);
  add((void **)&w.pos_of_atom, 4 * nn);
  add((void **)&w.atom_of_pos, 4 * rows);
  add((void **)&w.blk_counts, (size_t)4 * nblk * MAXT);
  add((void **)&w.type_count, 4 * MAXT);
  add((void **)&w.type_start, 4 * (MAXT + 1));
  add((void **)&w.rt, sizeof(double4) * nn * d.nnei);
  add((void **)&w.dr, sizeof(double4) * nn * d.nnei);
  if (!mixed) {
    add((void **)&w.T, sizeof(double) * nn * d.M1 * 4);
    add((void **)&w.D, sizeof(double) * rows * d.M1 * d.M2);
    add((void **)&w.dD, sizeof(double) * rows * d.M1 * d.M2);
    for (int l = 1; l <= d.n_fit; ++l) {
      add((void **)&w.Y[l], sizeof(double) * rows * d.fw[l]);
      add((void **)&w.Tt[l], sizeof(double) * rows * d.fw[l]);
      if (l < d.n_fit) add((void **)&w.G[l], sizeof(double) * rows * d.fw[l]);
    }
  } else {
    add((void **)&w.T32, sizeof(float) * nn * d.M1 * 4);
    add((void **)&w.D32, sizeof(float) * rows * d.M1 * d.M2);
    add((void **)&w.dD32, sizeof(float) * rows * d.M1 * d.M2);
    for (int l = 1; l <= d.n_fit; ++l) {
      add((void **)&w.Yf[l], sizeof(float) * rows * d.fw[l]);
      add((void **)&w.Ttf[l], sizeof(float) * rows * d.fw[l]);
      if (l < d.n_fit) add((void **)&w.Gf[l], sizeof(float) * rows * d.fw[l]);
    }
  }
  add((void **)&w.eatom, sizeof(double) * nn);
  add((void **)&w.partial, sizeof(double) * 1024);
  add((void **)&w.vir_part, sizeof(double) * 9 * 4096);
  add((void **)&w.force_tmp, sizeof(double) * 3 * nn);
  if (nd) add((void **)&w.net_deriv, sizeof(double) * 4 * nn * d.nnei);
  add((void **)&w.energy, sizeof(double) * 8);
  add((void **)&w.virial, sizeof(double) * 16);
  add((void **)&w.ke, sizeof(double) * 8);
  add((void **)&w.status, sizeof(DevStatus));
  for (auto &pr : plan) off += (pr.second + 255) / 256 * 256;
  void *base = nullptr;
  if (hipMalloc(&base, off) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, DP_E_OOM, "workspace allocation of " + std::to_string(off) + " bytes failed");
  }
  size_t o = 0;
  for (auto &pr : plan) {
    *pr.first = (char *)base + o;
    o += (pr.second + 255) / 256 * 256;
  }
  if (!nd) w.net_deriv = nullptr;
  w.G[0] = w.dD;
  w.Gf[0] = w.dD32;
  w.prec = c->precision;
  w.base = base;
  w.bytes = off;
  w.n_cap = nn;
  w.rows_cap = rows;
  w.ncell_cap = nc;
  w.cand_cap = cc;
  w.nd = nd;
  return DP_OK;
}

// ---------------------------------------------------------------------------
// device model
// ---------------------------------------------------------------------------
int upload_model(dp_ctx *c) {
  const HostModel &m = c->hm;
  Dims &d = c->dims;
  d = Dims{};
  d.ntypes = (int)m.ntypes;
  d.n_emb = (int)m.n_emb;
  d.n_fit = (int)m.n_fit;
  d.M1 = (int)m.emb_w[m.n_emb];
  d.M2 = (int)m.M2;
  d.rcut = m.rcut;
  d.rcut_smth = m.rcut_smth;
  d.inv_nc = 1.0 / m.desc_norm;
  d.off[0] = 0;
  for (int t = 0; t < d.ntypes; ++t) {
    d.sel[t] = (int)m.sel[t];
    d.off[t + 1] = d.off[t] + d.sel[t];
  }
  d.nnei = d.off[d.ntypes];
  for (int l = 0; l <= d.n_emb; ++l) {
    d.ew[l] = (int)m.emb_w[l];
    d.ekp[l] = rup(d.ew[l], 4);
    d.emp[l] = rup(d.ew[l], 16);
  }
  for (int l = 0; l <= d.n_fit + 1; ++l) d.fw[l] = (int)m.fit_w[l];
  if (d.M2 < 1 || d.M2 > 16 || d.M2 > d.M1) return fail(c, DP_E_MODEL, "M2 must be 1..16 and <= M1");
  for (int l = 1; l <= d.n_emb; ++l)
    if (d.emp[l] > 128) return fail(c, DP_E_MODEL, "embedding widths above 128 are not supported");
  if (!(d.rcut > 0 && d.rcut < 42.9)) return fail(c, DP_E_MODEL, "rcut must lie in (0, 42.9) A");
  if (!(d.rcut_smth >= 0 && d.rcut_smth < d.rcut)) return fail(c, DP_E_MODEL, "need 0 <= rcut_smth < rcut");
  if (!(m.desc_norm > 0)) return fail(c, DP_E_MODEL, "desc_norm must be positive");
  if (d.nnei < 1) return fail(c, DP_E_MODEL, "sum of sel must be positive");
  if (dpk::embed_lds_bytes(d, 1) > 65536 || dpk::embed_lds_bytes(d, 2) > 65536)
    return fail(c, DP_E_MODEL, "embedding net too wide for the per-wave LDS tiles");
  // embedding weights, padded
  std::vector<double> E;
  const int T = d.ntypes;
  for (int t = 0; t < T; ++t)
    for (int u = 0; u < T; ++u)
      for (int l = 0; l < d.n_emb; ++l) {
        const auto &W = m.eW[m.eidx(t, u, l)];
        const auto &b = m.eb[m.eidx(t, u, l)];
        const int in = d.ew[l], out = d.ew[l + 1];
        if (l == 0) {
          const int kp = d.ekp[1];
          c->eo.w[t][u][0] = (int64_t)E.size();
          E.resize(E.size() + kp, 0.0);
          for (int o = 0; o < out; ++o) E[c->eo.w[t][u][0] + o] = W[o];
          c->eo.b[t][u][0] = (int64_t)E.size();
          E.resize(E.size() + kp, 0.0);
          for (int o = 0; o < out; ++o) E[c->eo.b[t][u][0] + o] = b[o];
        } else {
          const int kp = d.ekp[l], mp = d.emp[l + 1];
          c->eo.w[t][u][l] = (int64_t)E.size();
          E.resize(E.size() + (size_t)kp * mp, 0.0);
          for (int i = 0; i < in; ++i)
            for (int o = 0; o < out; ++o) E[c->eo.w[t][u][l] + (size_t)i * mp + o] = W[(size_t)i * out + o];
          c->eo.b[t][u][l] = (int64_t)E.size();
          E.resize(E.size() + mp, 0.0);
          for (int o = 0; o < out; ++o) E[c->eo.b[t][u][l] + o] = b[o];
        }
      }
  std::vector<double> F;
  for (int t = 0; t < T; ++t)
    for (int l = 0; l <= d.n_fit; ++l) {
      c->fo.w[t][l] = (int64_t)F.size();
      const auto &W = m.fW[m.fidx(t, l)];
      F.insert(F.end(), W.begin(), W.end());
      c->fo.b[t][l] = (int64_t)F.size();
      const auto &b = m.fb[m.fidx(t, l)];
      F.insert(F.end(), b.begin(), b.end());
    }
  if (c->d_emb) (void)hipFree(c->d_emb);
  if (c->d_fit) (void)hipFree(c->d_fit);
  c->d_emb = c->d_fit = nullptr;
  HIPCHK(c, hipMalloc(&c->d_emb, sizeof(double) * E.size()));
  HIPCHK(c, hipMalloc(&c->d_fit, sizeof(double) * F.size()));
  HIPCHK(c, hipMemcpy(c->d_emb, E.data(), sizeof(double) * E.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_fit, F.data(), sizeof(double) * F.size(), hipMemcpyHostToDevice));
  return DP_OK;
}

// Mixed-precision weights: per (t,u) the LDS image of the embedding net, and
// for the fitting net 16-bit W^T / W for the first n16 layers plus f32 copies.
uint16_t h16_bits(double v, int prec) {
  const float f = (float)v;
  if (prec == 0) {
    _Float16 h = (_Float16)f;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
  }
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

int upload_mix(dp_ctx *c) {
  const HostModel &m = c->hm;
  const Dims &d = c->dims;
  const int prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  const int shape = mix_shape_id(d);
  if (shape < 0) return fail(c, DP_E_MODEL, "mixed precision supports embedding widths 25-50-100 and 16-32-100");
  if (mix_lds_bytes(shape, d.ntypes, 2) > 163840 || mix_lds_bytes(shape, d.ntypes, 1) > 163840)
    return fail(c, DP_E_MODEL, "too many atom types for the mixed-precision LDS layout");
  const int n16 = std::min(2, d.n_fit);
  for (int l = 0; l <= n16; ++l)
    if (d.fw[l] % 8 != 0) return fail(c, DP_E_MODEL, "16-bit fitting layers need widths divisible by 8");
  const size_t nb = mix_net_bytes(shape);
  const int T = d.ntypes;
  std::vector<unsigned char> nets(nb * T * T);
  for (int t = 0; t < T; ++t)
    for (int u = 0; u < T; ++u) {
      const double *W[3], *b[3];
      for (int l = 0; l < 3; ++l) {
        W[l] = m.eW[m.eidx(t, u, l)].data();
        b[l] = m.eb[m.eidx(t, u, l)].data();
      }
      mix_pack_net(shape, W, b, prec, nets.data() + (size_t)(t * T + u) * nb);
    }
  std::vector<unsigned char> F;
  auto align = [&]() { F.resize((F.size() + 255) / 256 * 256, 0); };
  FitMixOffsets fo{};
  for (int t = 0; t < T; ++t)
    for (int l = 0; l <= d.n_fit; ++l) {
      const auto &W = m.fW[m.fidx(t, l)];
      const auto &bb = m.fb[m.fidx(t, l)];
      const int in = d.fw[l], out = d.fw[l + 1];
      if (l < n16) {
        align();
        fo.wt16[t][l] = (int64_t)F.size();
        F.resize(F.size() + 2 * (size_t)in * out);
        uint16_t *wt = (uint16_t *)(F.data() + fo.wt16[t][l]);
        for (int i = 0; i < in; ++i)
          for (int o = 0; o < out; ++o) wt[(size_t)o * in + i] = h16_bits(W[(size_t)i * out + o], prec);
        align();
        fo.w16[t][l] = (int64_t)F.size();
        F.resize(F.size() + 2 * (size_t)in * out);
        uint16_t *wn = (uint16_t *)(F.data() + fo.w16[t][l]);
        for (size_t q = 0; q < (size_t)in * out; ++q) wn[q] = h16_bits(W[q], prec);
      }
      align();
      fo.w32[t][l] = (int64_t)F.size();
      F.resize(F.size() + 4 * (size_t)in * out);
      float *w32 = (float *)(F.data() + fo.w32[t][l]);
      for (size_t q = 0; q < (size_t)in * out; ++q) w32[q] = (float)W[q];
      align();
      fo.b32[t][l] = (int64_t)F.size();
      F.resize(F.size() + 4 * (size_t)out);
      float *b32 = (float *)(F.data() + fo.b32[t][l]);
      for (int o = 0; o < out; ++o) b32[o] = (float)bb[o];
    }
  if (c->d_mix_nets) (void)hipFree(c->d_mix_nets);
  if (c->d_fit_mix) (void)hipFree(c->d_fit_mix);
  c->d_mix_nets = c->d_fit_mix = nullptr;
  HIPCHK(c, hipMalloc(&c->d_mix_nets, nets.size()));
  HIPCHK(c, hipMalloc(&c->d_fit_mix, F.size()));
  HIPCHK(c, hipMemcpy(c->d_mix_nets, nets.data(), nets.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_fit_mix, F.data(), F.size(), hipMemcpyHostToDevice));
  c->fmo = fo;
  c->mix_shape = shape;
  c->n16 = n16;
  return DP_OK;
}

// ---------------------------------------------------------------------------
// one evaluation
// ---------------------------------------------------------------------------
int check_box(dp_ctx *c, const double *box, double rlist, double L[3]) {
  if (!box) return fail(c, DP_E_ARG, "box is NULL");
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (a != b && box[3 * a + b] != 0.0) return fail(c, DP_E_BOX, "only orthorhombic (diagonal) boxes are supported");
  for (int a = 0; a < 3; ++a) {
    L[a] = box[4 * a];
    if (!(L[a] > 2.0 * rlist) || !std::isfinite(L[a]))
      return fail(c, DP_E_BOX, "each box length must exceed 2*(rcut+skin) = " + std::to_string(2.0 * rlist));
  }
  return DP_OK;
}

CellGrid make_grid(const double L[3], double rlist) {
  CellGrid g{};
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = std::max(1, (int)std::floor(L[a] / rlist));
    g.side[a] = L[a] / g.nc[a];
    g.L[a] = L[a];
  }
  return g;
}

int cand_capacity(int64_t n, const double L[3], double rlist) {
  // twice the mean number of atoms within rlist, plus slack; never more than n
  const double rho = (double)n / (L[0] * L[1] * L[2]);
  const double expect = rho * 4.18879020478639 * rlist * rlist * rlist;
  const int64_t cap = std::min<int64_t>((int64_t)std::ceil(2.0 * expect + 64.0), std::max<int64_t>(n, 1));
  return rup((int)cap, 64);
}

constexpr int NMARK = 8;
constexpr int EV_MAX = 2048;

inline void tmark(dp_ctx *c, int k) {
  if (c->timing && c->nev < c->ev_cap) (void)hipEventRecord(c->ev[(size_t)c->nev * NMARK + k], c->stream);
}

inline void tnext(dp_ctx *c) {
  if (c->timing && c->nev < c->ev_cap) ++c->nev;
}

// Arguments of the embedding / fitting launches for the loaded policy.
EmbedArgs embed_args(dp_ctx *c, int64_t n, int64_t rows, double *F) {
  Workspace &w = c->ws;
  EmbedArgs ea{};
  ea.d = c->dims;
  ea.eo = c->eo;
  ea.ew = c->d_emb;
  ea.atom_of_pos = w.atom_of_pos;
  ea.pos_of_atom = w.pos_of_atom;
  ea.type_start = w.type_start;
  ea.rows = rows;
  ea.natoms = n;
  ea.xw = w.xw;
  ea.nlist = w.nlist;
  ea.nreal = w.nreal;
  ea.rt = w.rt;
  ea.dr = w.dr;
  ea.T = w.T;
  ea.D = w.D;
  ea.dD = w.dD;
  ea.force = F;
  ea.vir_part = w.vir_part;
  ea.net_deriv = c->keep ? w.net_deriv : nullptr;
  return ea;
}

FitArgs fit_args(dp_ctx *c, int64_t rows) {
  Workspace &w = c->ws;
  FitArgs fa{};
  fa.d = c->dims;
  fa.fo = c->fo;
  fa.fwt = c->d_fit;
  fa.type_start = w.type_start;
  fa.atom_of_pos = w.atom_of_pos;
  fa.rows = rows;
  fa.X0 = w.D;
  for (int l = 0; l <= MAXF; ++l) {
    fa.Y[l] = w.Y[l];
    fa.Tt[l] = w.Tt[l];
    fa.G[l] = w.G[l];
  }
  fa.eatom = w.eatom;
  return fa;
}

MixArgs mix_args(dp_ctx *c, int64_t rows, double *F) {
  Workspace &w = c->ws;
  MixArgs ma{};
  ma.d = c->dims;
  ma.shape = c->mix_shape;
  ma.prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  ma.nets = c->d_mix_nets;
  ma.rows = rows;
  ma.atom_of_pos = w.atom_of_pos;
  ma.xw = w.xw;
  ma.nlist = w.nlist;
  ma.nreal = w.nreal;
  ma.rt = w.rt;
  ma.dr = w.dr;
  ma.T32 = w.T32;
  ma.D32 = w.D32;
  ma.dD32 = w.dD32;
  ma.force = F;
  ma.vir_part = w.vir_part;
  ma.net_deriv = c->keep ? w.net_deriv : nullptr;
  return ma;
}

FitMixArgs fitmix_args(dp_ctx *c, int64_t rows) {
  Workspace &w = c->ws;
  FitMixArgs fa{};
  fa.d = c->dims;
  fa.fo = c->fmo;
  fa.w = c->d_fit_mix;
  fa.prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  fa.n16 = c->n16;
  fa.type_start = w.type_start;
  fa.atom_of_pos = w.atom_of_pos;
  fa.rows = rows;
  fa.X0 = w.D32;
  for (int l = 0; l <= MAXF; ++l) {
    fa.Y[l] = w.Yf[l];
    fa.Tt[l] = w.Ttf[l];
    fa.G[l] = w.Gf[l];
  }
  fa.eatom = w.eatom;
  return fa;
}

int64_t eval_rows(const dp_ctx *c, int64_t n) {
  return (n + ROW_TILE - 1) / ROW_TILE * ROW_TILE + (int64_t)ROW_TILE * c->dims.ntypes;
}

// Forward half of an evaluation: formatted list, environment matrix,
// embedding + descriptor, fitting net forward, energy.  Leaves everything
// the backward half needs in the workspace.
void eval_forward(dp_ctx *c, int64_t n, const double L[3]) {
  Workspace &w = c->ws;
  const Dims &d = c->dims;
  hipStream_t s = c->stream;
  const int64_t rows = eval_rows(c, n);
  tmark(c, 1);
  launch_format(s, n, w.xw, d, L, w.cand, w.cand_n, w.cand_cap, w.nlist, w.nreal, &w.status->overflow,
                w.status->max_real, &w.status->flags);
  tmark(c, 2);
  launch_env(s, n, w.xw, d, L, w.nlist, w.nreal, w.rt, w.dr);
  tmark(c, 3);
  if (c->precision == DP_FP64) {
    launch_embed_fwd_f64(s, embed_args(c, n, rows, nullptr));
    tmark(c, 4);
    launch_fit_f64(s, fit_args(c, rows), 1);
  } else {
    launch_embed_mix(s, mix_args(c, rows, nullptr), 1, mix_grid(rows));
    tmark(c, 4);
    launch_fit_mix(s, fitmix_args(c, rows), 1);
  }
  launch_sum(s, w.eatom, n, w.partial, w.energy, 1.0);
}

// Backward half (the adjoint): fitting net backward to dE/dD, then the
// embedding backward with the force and virial scatter into F.
void eval_backward(dp_ctx *c, int64_t n, double *F) {
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  const int64_t rows = eval_rows(c, n);
  if (c->precision == DP_FP64) {
    launch_fit_f64(s, fit_args(c, rows), 2);
    tmark(c, 5);
    launch_zero(s, F, 3 * n);
    const int grid = embed_bwd_grid(rows);
    tmark(c, 6);
    launch_embed_bwd_f64(s, embed_args(c, n, rows, F), grid);
    tmark(c, 7);
    launch_sum9(s, w.vir_part, grid, w.virial);
  } else {
    launch_fit_mix(s, fitmix_args(c, rows), 2);
    tmark(c, 5);
    launch_zero(s, F, 3 * n);
    const int grid = mix_grid(rows);
    tmark(c, 6);
    launch_embed_mix(s, mix_args(c, rows, F), 2, grid);
    tmark(c, 7);
    launch_sum9(s, w.vir_part, grid, w.virial);
  }
  tnext(c);
}

void eval_body(dp_ctx *c, int64_t n, const double L[3], double *F) {
  eval_forward(c, n, L);
  eval_backward(c, n, F);
}

void build_lists(dp_ctx *c, int64_t n, const CellGrid &g, double rlist, const uint32_t *cond) {
  Workspace &w = c->ws;
  launch_cells(c->stream, n, w.xw, g, w.cell_of, w.cell_start, w.cell_fill, w.cell_atoms, w.scan_tmp, cond);
  launch_candidates(c->stream, n, w.xw, g, w.cell_start, w.cell_atoms, rlist, w.cand_cap, w.cand, w.cand_n,
                    &w.status->flags, cond);
}

int read_status(dp_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->h_status, c->ws.status, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->stats.sel_overflow = (int64_t)c->h_status->overflow;
  for (int t = 0; t < MAXT; ++t) c->stats.max_real[t] = c->h_status->max_real[t];
  c->stats.nlist_builds = (int64_t)c->h_status->nbuild;
  return DP_OK;
}

__global__ void k_reset_status(DevStatus *st, uint32_t flags) {
  if (threadIdx.x == 0) {
    st->flags = flags;
    st->overflow = 0;
    for (int t = 0; t < MAXT; ++t) st->max_real[t] = 0;
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int dp_create(dp_ctx **out, int device, void *hip_stream) {
  if (!out) return DP_E_ARG;
  *out = nullptr;
  dp_ctx *c = new (std::nothrow) dp_ctx();
  if (!c) return DP_E_OOM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return DP_E_HIP;
  }
  if (hipHostMalloc((void **)&c->h_status, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return DP_E_HIP;
  }
  *out = c;
  return DP_OK;
}

void dp_destroy(dp_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_ws(c->ws);
  if (c->d_emb) (void)hipFree(c->d_emb);
  if (c->d_fit) (void)hipFree(c->d_fit);
  if (c->d_mix_nets) (void)hipFree(c->d_mix_nets);
  if (c->d_fit_mix) (void)hipFree(c->d_fit_mix);
  if (c->h_status) (void)hipHostFree(c->h_status);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char *dp_last_error(const dp_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

int dp_set_model(dp_ctx *c, const void *blob, size_t nbytes, int precision) {
  if (!c || !blob) return fail(c, DP_E_ARG, "NULL argument");
  if (precision != DP_FP64 && precision != DP_MIX_FP16 && precision != DP_MIX_BF16)
    return fail(c, DP_E_ARG, "unsupported precision policy");
  HIPCHK(c, hipSetDevice(c->device));
  HostModel m;
  std::string err;
  if (!parse_blob(blob, nbytes, m, err)) return fail(c, DP_E_MODEL, err);
  c->hm = std::move(m);
  free_ws(c->ws);
  c->has_model = false;
  int rc = upload_model(c);
  if (rc) return rc;
  c->precision = precision;
  if (precision != DP_FP64) {
    rc = upload_mix(c);
    if (rc) return rc;
  }
  c->has_model = true;
  return DP_OK;
}

int dp_set_precision(dp_ctx *c, int precision) {
  if (!c) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "no model");
  if (precision != DP_FP64 && precision != DP_MIX_FP16 && precision != DP_MIX_BF16)
    return fail(c, DP_E_ARG, "unsupported precision policy");
  const int old = c->precision;
  c->precision = precision;
  if (precision != DP_FP64) {
    int rc = upload_mix(c);
    if (rc) {
      c->precision = old;
      return rc;
    }
  }
  return DP_OK;
}

int dp_keep_intermediates(dp_ctx *c, int keep) {
  if (!c) return DP_E_ARG;
  c->keep = keep != 0;
  return DP_OK;
}

int dp_enable_timing(dp_ctx *c, int on) {
  if (!c) return DP_E_ARG;
  if (on && c->ev.empty()) {
    c->ev.resize((size_t)EV_MAX * NMARK, nullptr);
    for (auto &e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(c, DP_E_HIP, "hipEventCreate failed");
    c->ev_cap = EV_MAX;
  }
  c->timing = on != 0;
  c->nev = 0;
  return DP_OK;
}

int dp_get_timing(dp_ctx *c, const char *name, double *ms) {
  if (!c || !name || !ms) return DP_E_ARG;
  // marks: 0 start, 1 lists built, 2 format, 3 env, 4 embed_fwd, 5 fitting
  // net, 6 energy sum + force clear, 7 embed_bwd (with forces and virial)
  static const char *names[] = {"lists", "format", "env", "embed_fwd", "fit", "embed_bwd", "total"};
  static const int from[] = {0, 1, 2, 3, 4, 6, 0};
  static const int to[] = {1, 2, 3, 4, 5, 7, 7};
  if (c->nev == 0) return fail(c, DP_E_ARG, "no timed evaluation");
  for (int k = 0; k < 7; ++k)
    if (std::strcmp(name, names[k]) == 0) {
      double sum = 0.0;
      for (int64_t e = 0; e < c->nev; ++e) {
        float v = 0.f;
        hipEvent_t a = c->ev[(size_t)e * NMARK + from[k]], b = c->ev[(size_t)e * NMARK + to[k]];
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&v, a, b) != hipSuccess) {
          (void)hipGetLastError();
          return fail(c, DP_E_ARG, "timing events incomplete");
        }
        sum += v;
      }
      *ms = sum / (double)c->nev;
      return DP_OK;
    }
  return fail(c, DP_E_ARG, "unknown timer name");
}

static int compute_impl(dp_ctx *c, int64_t n, const double *coords, const int32_t *types, const double *box,
                        double *energy, double *forces, double *virial, bool backward) {
  if (!c) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "evaluation before dp_set_model");
  if (n < 0 || n >= (1 << 26)) return fail(c, DP_E_ARG, "natoms must be in [0, 2^26)");
  if (n > 0 && (!coords || !types)) return fail(c, DP_E_ARG, "NULL coords or types");
  HIPCHK(c, hipSetDevice(c->device));
  const Dims &d = c->dims;
  double L[3];
  const double rlist = d.rcut;
  int rc = check_box(c, box, rlist, L);
  if (rc) return rc;
  hipStream_t s = c->stream;
  CellGrid g = make_grid(L, rlist);
  const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
  int cap = cand_capacity(n, L, rlist);
  c->fwd_ready = false;
  for (int attempt = 0; attempt < 4; ++attempt) {
    rc = ensure_ws(c, std::max<int64_t>(n, 1), ncell, cap);
    if (rc) return rc;
    Workspace &w = c->ws;
    double *F = forces ? forces : w.force_tmp;
    tmark(c, 0);
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, w.status, 0u);
    if (n > 0) {
      launch_wrap(s, n, coords, types, d.ntypes, L, w.xw, &w.status->flags);
      launch_type_sort(s, n, w.xw, d.ntypes, w.blk_counts, w.type_count, w.type_start, w.pos_of_atom,
                       w.atom_of_pos, w.rows_cap);
      build_lists(c, n, g, rlist, nullptr);
      eval_forward(c, n, L);
      if (backward) eval_backward(c, n, F);
    } else {
      launch_zero(s, w.energy, 1);
      launch_zero(s, w.virial, 9);
      for (int k = 1; k < NMARK; ++k) tmark(c, k);
      tnext(c);
    }
    if (energy) HIPCHK(c, hipMemcpyAsync(energy, w.energy, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (virial && backward)
      HIPCHK(c, hipMemcpyAsync(virial, w.virial, 9 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipGetLastError());
    rc = read_status(c);
    if (rc) return rc;
    const uint32_t fl = c->h_status->flags;
    if (fl & FLAG_BAD_TYPE) return fail(c, DP_E_TYPE, "atom type out of range");
    if (fl & FLAG_KEY_CAP) return fail(c, DP_E_CAP, "more than 1024 neighbours within rcut of one atom");
    if (fl & FLAG_CAND_CAP) {
      cap *= 2;
      if (c->timing && c->nev > 0) --c->nev;
      continue;
    }
    c->stats.natoms = n;
    c->stats.evaluations += 1;
    c->stats.cand_cap = c->ws.cand_cap;
    c->last_n = n;
    c->fwd_ready = !backward;
    return DP_OK;
  }
  return fail(c, DP_E_CAP, "candidate list capacity could not be sized");
}

__global__ void k_scale(double *x, int64_t n, double a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= a;
}

int dp_compute(dp_ctx *c, int64_t n, const double *coords, const int32_t *types, const double *box, double *energy,
               double *forces, double *virial) {
  return compute_impl(c, n, coords, types, box, energy, forces, virial, true);
}

int dp_energy(dp_ctx *c, int64_t n, const double *coords, const int32_t *types, const double *box, double *energy) {
  return compute_impl(c, n, coords, types, box, energy, nullptr, nullptr, false);
}

int dp_energy_backward(dp_ctx *c, double grad_energy, double *forces, double *virial) {
  if (!c) return DP_E_ARG;
  if (!c->fwd_ready) return fail(c, DP_E_ARG, "dp_energy_backward needs a preceding dp_energy");
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t n = c->last_n;
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  double *F = forces ? forces : w.force_tmp;
  if (n > 0) {
    tmark(c, 0);
    tmark(c, 1);
    tmark(c, 2);
    tmark(c, 3);
    tmark(c, 4);
    eval_backward(c, n, F);
    if (grad_energy != 1.0) {
      hipLaunchKernelGGL(k_scale, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, F, 3 * n, grad_energy);
      hipLaunchKernelGGL(k_scale, dim3(1), dim3(64), 0, s, w.virial, (int64_t)9, grad_energy);
    }
  } else {
    launch_zero(s, w.virial, 9);
  }
  if (virial) HIPCHK(c, hipMemcpyAsync(virial, w.virial, 9 * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipGetLastError());
  return DP_OK;
}

int dp_get_nlist(dp_ctx *c, int32_t *nlist, int32_t *nreal) {
  if (!c || (!nlist && !nreal)) return DP_E_ARG;
  if (!c->has_model || c->ws.n_cap < 0) return fail(c, DP_E_NOMODEL, "no evaluation yet");
  const int64_t n = c->last_n;
  if (nlist)
    HIPCHK(c, hipMemcpyAsync(nlist, c->ws.nlist, sizeof(int32_t) * n * c->dims.nnei, hipMemcpyDeviceToDevice,
                             c->stream));
  if (nreal)
    HIPCHK(c, hipMemcpyAsync(nreal, c->ws.nreal, sizeof(int32_t) * n * c->dims.ntypes, hipMemcpyDeviceToDevice,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return DP_OK;
}

int dp_get_intermediates(dp_ctx *c, double *atom_e, double *T, double *D, double *net_deriv) {
  if (!c) return DP_E_ARG;
  if (!c->has_model || c->ws.n_cap < 0) return fail(c, DP_E_NOMODEL, "no evaluation yet");
  const int64_t n = c->last_n;
  const Dims &d = c->dims;
  hipStream_t s = c->stream;
  if ((T || D) && c->precision != DP_FP64)
    return fail(c, DP_E_ARG, "T and D intermediates are kept in double only under DP_FP64");
  if (atom_e) HIPCHK(c, hipMemcpyAsync(atom_e, c->ws.eatom, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (T) HIPCHK(c, hipMemcpyAsync(T, c->ws.T, sizeof(double) * n * d.M1 * 4, hipMemcpyDeviceToDevice, s));
  if (D || net_deriv) {
    std::vector<int32_t> pos(n > 0 ? n : 1);
    HIPCHK(c, hipMemcpyAsync(pos.data(), c->ws.pos_of_atom, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const size_t MM = (size_t)d.M1 * d.M2;
    if (D)
      for (int64_t i = 0; i < n; ++i)
        HIPCHK(c, hipMemcpyAsync(D + i * MM, c->ws.D + (size_t)pos[i] * MM, sizeof(double) * MM,
                                 hipMemcpyDeviceToDevice, s));
    if (net_deriv) {
      if (!c->ws.net_deriv) return fail(c, DP_E_ARG, "net_deriv needs dp_keep_intermediates(c,1) before dp_compute");
      // only the real slots of each row are written by the kernels
      HIPCHK(c, hipMemcpyAsync(net_deriv, c->ws.net_deriv, sizeof(double) * 4 * n * d.nnei, hipMemcpyDeviceToDevice,
                               s));
    }
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return DP_OK;
}

int dp_get_stats(dp_ctx *c, dp_stats *out) {
  if (!c || !out) return DP_E_ARG;
  *out = c->stats;
  return DP_OK;
}

int dp_md_run(dp_ctx *c, int64_t n, double *coords, double *vel, const int32_t *types, const double *box,
              const double *masses, double dt, double skin, int64_t nsteps, int64_t thermo_every, double *thermo,
              double *forces) {
  if (!c) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "no model");
  if (n < 1 || n >= (1 << 26) || !coords || !vel || !types || !masses || nsteps < 0 || !(skin >= 0) || !(dt > 0))
    return fail(c, DP_E_ARG, "bad MD arguments");
  if (thermo && thermo_every < 1) return fail(c, DP_E_ARG, "thermo_every must be >= 1");
  HIPCHK(c, hipSetDevice(c->device));
  c->fwd_ready = false;
  const Dims &d = c->dims;
  const double rlist = d.rcut + skin;
  double L[3];
  int rc = check_box(c, box, rlist, L);
  if (rc) return rc;
  hipStream_t s = c->stream;
  CellGrid g = make_grid(L, rlist);
  const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
  const int cap = cand_capacity(n, L, rlist);
  rc = ensure_ws(c, n, ncell, cap);
  if (rc) return rc;
  Workspace &w = c->ws;
  double *F = forces ? forces : w.force_tmp;
  double inv_m[MAXT] = {0}, mass[MAXT] = {0};
  for (int t = 0; t < d.ntypes; ++t) {
    if (!(masses[t] > 0)) return fail(c, DP_E_ARG, "masses must be positive");
    mass[t] = masses[t];
    inv_m[t] = 1.0 / (masses[t] * MVV2E);
  }
  const double ndof_kb = (3.0 * n - 3.0) * KB_EV;
  const double inv3v = 1.0 / (3.0 * L[0] * L[1] * L[2]);
  int64_t row = 0;
  tmark(c, 0);
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, w.status, (uint32_t)FLAG_REBUILD);
  launch_wrap(s, n, coords, types, d.ntypes, L, w.xw, &w.status->flags);
  launch_type_sort(s, n, w.xw, d.ntypes, w.blk_counts, w.type_count, w.type_start, w.pos_of_atom, w.atom_of_pos,
                   w.rows_cap);
  build_lists(c, n, g, rlist, &w.status->flags);
  launch_copy_ref(s, n, w.xw, w.xref, &w.status->flags);
  launch_end_rebuild(s, &w.status->flags, &w.status->nbuild);
  eval_body(c, n, L, F);
  if (thermo) {
    launch_kinetic(s, n, vel, types, mass, w.partial, w.ke);
    launch_thermo_row(s, thermo + 6 * row++, 0.0, w.ke, w.energy, w.virial, ndof_kb, inv3v, &w.status->flags);
  }
  for (int64_t st = 1; st <= nsteps; ++st) {
    tmark(c, 0);
    launch_verlet_half(s, n, vel, F, types, inv_m, 0.5 * dt);
    launch_verlet_drift(s, n, coords, vel, dt, L);
    launch_wrap(s, n, coords, types, d.ntypes, L, w.xw, &w.status->flags);
    launch_max_disp(s, n, w.xw, w.xref, L, 0.5 * skin, &w.status->flags);
    build_lists(c, n, g, rlist, &w.status->flags);
    launch_copy_ref(s, n, w.xw, w.xref, &w.status->flags);
    launch_end_rebuild(s, &w.status->flags, &w.status->nbuild);
    eval_body(c, n, L, F);
    launch_verlet_half(s, n, vel, F, types, inv_m, 0.5 * dt);
    const bool th = thermo && (st % thermo_every == 0);
    if (th) {
      launch_kinetic(s, n, vel, types, mass, w.partial, w.ke);
      launch_thermo_row(s, thermo + 6 * row++, (double)st, w.ke, w.energy, w.virial, ndof_kb, inv3v,
                        &w.status->flags);
    }
    if (th || st == nsteps) {
      HIPCHK(c, hipGetLastError());
      rc = read_status(c);
      if (rc) return rc;
      const uint32_t fl = c->h_status->flags;
      if (fl & FLAG_BAD_TYPE) return fail(c, DP_E_TYPE, "atom type out of range");
      if (fl & FLAG_KEY_CAP) return fail(c, DP_E_CAP, "more than 1024 neighbours within rcut of one atom");
      if (fl & FLAG_CAND_CAP) return fail(c, DP_E_CAP, "skin candidate list overflow; use a smaller skin");
      if (fl & FLAG_NONFINITE) return fail(c, DP_E_NONFINITE, "non-finite energy at step " + std::to_string(st));
    }
    c->stats.evaluations += 1;
  }
  if (nsteps == 0) {
    rc = read_status(c);
    if (rc) return rc;
  }
  c->stats.natoms = n;
  c->stats.cand_cap = c->ws.cand_cap;
  c->last_n = n;
  return DP_OK;
}

}  // extern "C"
