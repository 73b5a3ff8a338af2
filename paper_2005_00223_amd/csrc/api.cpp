// Host runtime of the C ABI declared in include/dpmi.h: model-blob parsing,
// device weight layout, the workspace arena (allocated once, grown only when
// a larger system arrives -- the paper's "trunk of GPU memory", Section
// V-B), and the launch sequence of one evaluation and of the MD loop.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dp_internal.h"
#include "dp_mix.h"
#include "dp_wide.h"
#include "dp_student.h"
#include "dpmi.h"

using namespace dpk;

namespace dpk {
size_t embed_lds_bytes(const Dims &d, int pass);
}

// Workspace of the no-allocation entry point (dp_compute_noalloc): a static
// device array, one copy per GPU, held until the process ends.  Host code
// never hands this name to a kernel or a copy (on the host it is only a
// stand-in); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current (scratch_address).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[SCRATCH_DEVICES];
void *g_scratch_ptr[SCRATCH_DEVICES];
hipError_t g_scratch_rc[SCRATCH_DEVICES];

// Device address of `scratch` on `device`, which must be the current device.
// NULL (and the HIP error in *rc) when the lookup failed.
void *scratch_address(int device, hipError_t *rc) {
  if (device < 0 || device >= SCRATCH_DEVICES) {
    *rc = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void *p = nullptr;
    g_scratch_rc[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g_scratch_rc[device] != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_scratch_ptr[device] = p;
    g_scratch_done[device] = true;
  }
  *rc = g_scratch_rc[device];
  return g_scratch_ptr[device];
}
}  // namespace

namespace {

constexpr double MVV2E = 103.642696562;
constexpr double KB_EV = 8.617333262e-5;

// ---------------------------------------------------------------------------
// model blob
// ---------------------------------------------------------------------------
struct HostModel {
  int64_t ntypes = 0, n_emb = 0, n_fit = 0, M2 = 0;
  int64_t emb_lin = 0;  // 1: affine last embedding layer
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
  if (!r.i64(version) || (version != 1 && version != 2)) return err = "blob: unsupported version", false;
  if (!r.i64(m.ntypes) || !r.i64(m.n_emb) || !r.i64(m.n_fit) || !r.i64(m.M2)) return err = "blob: truncated header", false;
  m.emb_lin = 0;
  if (version == 2 && (!r.i64(m.emb_lin) || (m.emb_lin != 0 && m.emb_lin != 1)))
    return err = "blob: bad emb_out_linear flag", false;
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
  double judge_rmse;   // force RMSE of the last student judge
  double judge_count;  // atoms it covered
  int32_t sub_rows;    // padded rows of the judge's atom subset
  uint32_t smax_bits;  // largest s of the frame (float bits), for the student table
  uint32_t defer_count;  // nets the table backward left to the layers
  long long fault_step;  // MD: the step an error flag stopped the integrator at (-1: none)
};

struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
  int64_t n_cap = -1, rows_cap = 0, ncell_cap = 0;
  int cand_cap = 0;
  bool nd = false;
  bool owned = true;  // base came from hipMalloc (false: the static scratch array)
  double4 *xw = nullptr, *xref = nullptr, *rt = nullptr, *dr = nullptr;
  float4 *rt32 = nullptr;  // mixed precision: the environment matrix in FP32
  int32_t *cell_of, *cell_atoms, *cell_start, *cell_fill, *scan_tmp, *cand, *cand_n, *nlist, *nreal, *pos_of_atom,
      *atom_of_pos, *blk_counts, *type_count, *type_start, *defer;
  double *T, *D, *dD, *Y[MAXF + 1], *Tt[MAXF + 1], *G[MAXF + 1], *eatom, *partial, *vir_part, *force_tmp,
      *net_deriv, *energy, *virial, *ke;
  // student judge: teacher forces / energy / virial, RMSE partial sums,
  // sampled-judge region marks and its type-padded row set
  double *force_j, *energy_j, *virial_j, *rmse_part;
  int32_t *judge_mark, *sub_atom_of_pos, *sub_type_count, *sub_type_start, *sub_blk;
  // cell-ordered force scatter: per-atom cell codes, per-cell force parts [27][n][3]
  uint32_t *cell_code;
  double *cell_part;
  // mixed-precision buffers
  float *T32, *dT32, *tbuf;
  int prec = -1;  // precision the buffers were laid out for
  DevStatus *status;
};

}  // namespace

// Student training state (buffers for one Adam batch per net).
struct Student {
  int nets = 0, M1 = 0, np = 0;
  int64_t cap = 0;       // samples per net of one batch the per-batch buffers hold
  int64_t cap_draw = 0;  // samples per net one draw (several batches) can hold
  void *base = nullptr;
  float *params = nullptr, *m = nullptr, *v = nullptr, *gpart = nullptr, *wt = nullptr, *gout = nullptr;
  double *lpart = nullptr, *s = nullptr, *G = nullptr, *lspart = nullptr, *lsfold = nullptr, *X = nullptr, *chk = nullptr,
         *loss = nullptr;
  int32_t *status = nullptr;
  bool have_params = false;
  int64_t t = 0;  // Adam steps taken since initialisation
};

// One set of embedding nets (the teacher's, or the student's) on the device.
struct EmbNets {
  Dims d{};                         // model dims with this set's embedding widths
  EmbOffsets eo{};
  double *d_emb = nullptr;          // FP64 padded weights
  float *d_emb32 = nullptr;         // the same rounded to FP32 (DP_MIX_FP32)
  unsigned char *d_mix = nullptr;   // mixed-precision LDS images
  int mix_shape = -1;
  float *d_tab = nullptr;           // tabulated second layer (student nets, mixed precision)
  unsigned char *d_wide = nullptr;  // wide nets (mixed precision): packed GEMM weights
  WideNet wnet[WIDE_NETS]{};        // their per-net offsets
  bool wide = false;
  double tab_shi = 0.0;             // its range of s
  bool tab_ok = false;
  bool ready = false;
};

struct dp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool has_model = false;
  int precision = DP_FP64;
  HostModel hm;                     // teacher
  Dims dims{};                      // teacher dims (geometry, fitting net)
  FitOffsets fo{};
  double *d_fit = nullptr;
  float *d_fit32 = nullptr;         // fitting weights rounded to FP32 (DP_MIX_FP32)
  // mixed-precision fitting weights (16-bit MFMA operands + f32)
  unsigned char *d_fit_mix = nullptr;
  FitMixOffsets fmo{};
  int n16 = 0;
  EmbNets en[2];                    // [0] teacher, [1] student
  int active = 0;                   // embedding set used by evaluations
  CellGrid cgrid{};                 // grid of the last cell-list build
  double box_L[3] = {0.0, 0.0, 0.0};  // box lengths of the last lists
  bool cgrid_ok = false;
  int scatter = 0;                  // dp_set_force_scatter mode
  bool use_tab = true;              // dp_student_table
  HostModel shm;                    // student (embedding part; fitting = teacher's)
  Student *st = nullptr;            // student training state
  int64_t judge_every = 20;         // MD judge period (0 = off)
  double judge_max = 1e-3;          // eV/A
  double judge_side = 0.0;          // > 0: judge the atoms of a cube of this side (A)
  // row set of the evaluation when it is not the full one (sampled judge)
  const int32_t *ov_atom_of_pos = nullptr, *ov_type_start = nullptr;
  int64_t ov_rows = 0;
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
  // wide embedding path: pair offsets, per-net counts, two activation buffers
  struct {
    int32_t *poff = nullptr, *cnt = nullptr;
    int64_t n_cap = 0;
    uint16_t *X[2] = {nullptr, nullptr};
    size_t x_cap = 0;  // elements per activation buffer
    int64_t row0[WIDE_NETS + 1]{};
    int32_t cnt_h[WIDE_NETS]{};
    int out = 0;       // buffer holding G after the forward
    int split = 1;     // activation storage the forward laid the rows out with
    bool ok = false;   // the forward of this evaluation ran
  } wb;
  int pending_rc = DP_OK;  // an error inside an evaluation (reported by read_status)
  int wide_split = 1;      // wide nets: activations stored as hi + lo 16-bit halves (0: one 16-bit value)
  // no-allocation entry point: the device address of this GPU's static
  // scratch array (NULL if its lookup failed, scratch_rc says why), the
  // workspace laid out on it, and whether an evaluation runs on it now
  // local (brick + ghost shell) evaluation: atoms the forces cover, when
  // more than the centres (0: the centres are all atoms)
  int64_t n_force = 0;
  void *scratch = nullptr;
  hipError_t scratch_rc = hipSuccess;
  Workspace ws_na;
  bool noalloc = false;
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
  if (w.base && w.owned) (void)hipFree(w.base);
  w = Workspace{};
}

void free_wide(dp_ctx *c) {
  for (void *p : {(void *)c->wb.poff, (void *)c->wb.X[0], (void *)c->wb.X[1]})
    if (p) (void)hipFree(p);
  c->wb.poff = c->wb.cnt = nullptr;
  c->wb.X[0] = c->wb.X[1] = nullptr;
  c->wb.n_cap = 0;
  c->wb.x_cap = 0;
  c->wb.ok = false;
}

void free_student(dp_ctx *c) {
  if (!c->st) return;
  if (c->st->base) (void)hipFree(c->st->base);
  delete c->st;
  c->st = nullptr;
}

// Precision policies: DP_FP64 and DP_MIX_FP32 run the FP64-structured
// kernels (in double and in float), DP_MIX_FP16 / DP_MIX_BF16 the
// register-resident 16-bit kernels.
inline bool prec16(int p) { return p == DP_MIX_FP16 || p == DP_MIX_BF16; }
inline bool prec_ok(int p) { return p == DP_FP64 || p == DP_MIX_FP32 || prec16(p); }

// Lay every buffer of the workspace out in one block: returns the block's
// size for nn atoms, nc cells and cc candidate slots per atom, and, when
// base is not NULL, points the buffers of w into the block at base.
size_t ws_carve(const dp_ctx *c, Workspace &w, int64_t nn, int64_t nc, int cc, bool nd, char *base) {
  const Dims &d = c->dims;
  const bool mixed = prec16(c->precision);
  const bool f32 = c->precision == DP_MIX_FP32;
  const size_t rb = f32 ? sizeof(float) : sizeof(double);  // FP64-structured buffers
  const int64_t rows = (nn + ROW_TILE - 1) / ROW_TILE * ROW_TILE + (int64_t)ROW_TILE * d.ntypes;
  const int64_t nblk = (nn + 255) / 256 + 1;
  size_t off = 0;
  auto add = [&](void **p, size_t bytes) {
    if (base) *p = base + off;
    off += (bytes + 255) / 256 * 256;
  };
  add((void **)&w.xw, sizeof(double4) * nn);
  add((void **)&w.xref, sizeof(double4) * nn);
  add((void **)&w.cell_of, 4 * nn);
  add((void **)&w.cell_atoms, 4 * nn);
  add((void **)&w.cell_code, 4 * nn);
  if (mixed) add((void **)&w.cell_part, sizeof(double) * 81 * nn);
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
  if (mixed || f32) add((void **)&w.rt32, sizeof(float4) * nn * d.nnei);
  else add((void **)&w.rt, sizeof(double4) * nn * d.nnei);
  if (!mixed) add((void **)&w.dr, sizeof(double4) * nn * d.nnei);
  if (!mixed) {
    // in float under DP_MIX_FP32 (the pointers are then read as float)
    add((void **)&w.T, rb * nn * d.M1 * 4);
    add((void **)&w.D, rb * rows * d.M1 * d.M2);
    add((void **)&w.dD, rb * rows * d.M1 * d.M2);
    for (int l = 1; l <= d.n_fit; ++l) {
      add((void **)&w.Y[l], rb * rows * d.fw[l]);
      add((void **)&w.Tt[l], rb * rows * d.fw[l]);
      if (l < d.n_fit) add((void **)&w.G[l], rb * rows * d.fw[l]);
    }
  } else {
    add((void **)&w.T32, sizeof(float) * nn * d.M1 * 4);
    add((void **)&w.dT32, sizeof(float) * nn * d.M1 * 4);
    add((void **)&w.tbuf, sizeof(float) * fit_mix_tbuf_floats(d, rows));
    add((void **)&w.defer, (size_t)4 * nn * d.ntypes);
  }
  add((void **)&w.eatom, sizeof(double) * nn);
  add((void **)&w.partial, sizeof(double) * 1024);
  add((void **)&w.vir_part, sizeof(double) * 9 * 4096);
  add((void **)&w.force_tmp, sizeof(double) * 3 * nn);
  if (nd) add((void **)&w.net_deriv, sizeof(double) * 4 * nn * d.nnei);
  add((void **)&w.energy, sizeof(double) * 8);
  add((void **)&w.virial, sizeof(double) * 16);
  add((void **)&w.ke, sizeof(double) * 8);
  add((void **)&w.force_j, sizeof(double) * 3 * nn);
  add((void **)&w.energy_j, sizeof(double) * 8);
  add((void **)&w.virial_j, sizeof(double) * 16);
  add((void **)&w.rmse_part, sizeof(double) * 512);
  add((void **)&w.judge_mark, 4 * nn);
  add((void **)&w.sub_atom_of_pos, 4 * rows);
  add((void **)&w.sub_type_count, 4 * MAXT);
  add((void **)&w.sub_type_start, 4 * (MAXT + 1));
  add((void **)&w.sub_blk, (size_t)4 * nblk * MAXT);
  add((void **)&w.status, sizeof(DevStatus));
  if (base) {
    if (!nd) w.net_deriv = nullptr;
    if (!mixed) {
      w.cell_part = nullptr;
      w.defer = nullptr;
    }
    if (mixed) w.rt = w.dr = nullptr;
    else if (f32) w.rt = nullptr;
    else w.rt32 = nullptr;
    w.G[0] = w.dD;
    w.prec = c->precision;
    w.base = base;
    w.bytes = off;
    w.n_cap = nn;
    w.rows_cap = rows;
    w.ncell_cap = nc;
    w.cand_cap = cc;
    w.nd = nd;
  }
  return off;
}

// Make the workspace hold n atoms, ncell cells and cand_cap candidates per
// atom.  Normally one allocation, grown by a quarter beyond the need; in
// the no-allocation entry point the block is the device's static scratch
// array instead, laid out for exactly this call (an error if too small).
int ensure_ws(dp_ctx *c, int64_t n, int64_t ncell, int cand_cap) {
  Workspace &w = c->ws;
  const bool need_nd = c->keep;
  if (n <= w.n_cap && ncell <= w.ncell_cap && cand_cap <= w.cand_cap && (!need_nd || w.nd) &&
      w.prec == c->precision)
    return DP_OK;
  if (c->noalloc) {
    Workspace nw{};
    const size_t need = ws_carve(c, nw, n, ncell, cand_cap, need_nd, nullptr);
    if (need > NOALLOC_SCRATCH_BYTES)
      return fail(c, DP_E_CAP, "dp_compute_noalloc: this system needs a workspace of " + std::to_string(need) +
                                   " bytes, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                   "-byte static scratch holds (use dp_compute)");
    nw.owned = false;
    ws_carve(c, nw, n, ncell, cand_cap, need_nd, (char *)c->scratch);
    w = nw;
    c->cgrid_ok = false;
    return DP_OK;
  }
  int64_t nn = std::max<int64_t>(n, w.n_cap > 0 ? (w.n_cap * 5) / 4 : n);
  nn = std::max<int64_t>(nn, 1);
  int64_t nc = std::max<int64_t>(ncell, w.ncell_cap);
  int cc = std::max(cand_cap, w.cand_cap);
  bool nd = need_nd || w.nd;
  free_ws(w);
  Workspace nw{};
  const size_t off = ws_carve(c, nw, nn, nc, cc, nd, nullptr);
  void *base = nullptr;
  if (hipMalloc(&base, off) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, DP_E_OOM, "workspace allocation of " + std::to_string(off) + " bytes failed");
  }
  ws_carve(c, nw, nn, nc, cc, nd, (char *)base);
  w = nw;
  c->cgrid_ok = false;
  return DP_OK;
}

// ---------------------------------------------------------------------------
// device model
// ---------------------------------------------------------------------------
// Embedding dims of model m on top of the teacher dims c->dims.
int emb_dims(dp_ctx *c, const HostModel &m, Dims &d) {
  d = c->dims;
  d.n_emb = (int)m.n_emb;
  d.emb_lin = (int)m.emb_lin;
  for (int l = 0; l <= MAXL; ++l) d.ew[l] = d.ekp[l] = d.emp[l] = 0;
  for (int l = 0; l <= d.n_emb; ++l) {
    d.ew[l] = (int)m.emb_w[l];
    d.ekp[l] = rup(d.ew[l], 4);
    d.emp[l] = rup(d.ew[l], 16);
  }
  if (d.ew[d.n_emb] != d.M1) return fail(c, DP_E_MODEL, "embedding output width must equal M1");
  for (int l = 1; l <= d.n_emb; ++l)
    if (d.ew[l] > 2048) return fail(c, DP_E_MODEL, "embedding widths above 2048 are not supported");
  return DP_OK;
}

// Whether the FP64 embedding kernels take these widths (per-wave LDS tiles).
bool f64_emb_ok(const Dims &d, const char **why) {
  for (int l = 1; l <= d.n_emb; ++l)
    if (d.emp[l] > 128) return *why = "FP64 embedding kernels take widths up to 128 (wider nets: mixed precision)", false;
  if (dpk::embed_lds_bytes(d, 1) > 65536 || dpk::embed_lds_bytes(d, 2) > 65536)
    return *why = "embedding net too wide for the per-wave LDS tiles", false;
  return true;
}

// FP64 padded embedding weights of model m into en.
int upload_emb(dp_ctx *c, const HostModel &m, EmbNets &en) {
  int rc = emb_dims(c, m, en.d);
  if (rc) return rc;
  const Dims &d = en.d;
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
          en.eo.w[t][u][0] = (int64_t)E.size();
          E.resize(E.size() + kp, 0.0);
          for (int o = 0; o < out; ++o) E[en.eo.w[t][u][0] + o] = W[o];
          en.eo.b[t][u][0] = (int64_t)E.size();
          E.resize(E.size() + kp, 0.0);
          for (int o = 0; o < out; ++o) E[en.eo.b[t][u][0] + o] = b[o];
        } else {
          const int kp = d.ekp[l], mp = d.emp[l + 1];
          en.eo.w[t][u][l] = (int64_t)E.size();
          E.resize(E.size() + (size_t)kp * mp, 0.0);
          for (int i = 0; i < in; ++i)
            for (int o = 0; o < out; ++o) E[en.eo.w[t][u][l] + (size_t)i * mp + o] = W[(size_t)i * out + o];
          en.eo.b[t][u][l] = (int64_t)E.size();
          E.resize(E.size() + mp, 0.0);
          for (int o = 0; o < out; ++o) E[en.eo.b[t][u][l] + o] = b[o];
        }
      }
  if (en.d_emb) (void)hipFree(en.d_emb);
  if (en.d_emb32) (void)hipFree(en.d_emb32);
  en.d_emb = nullptr;
  en.d_emb32 = nullptr;
  HIPCHK(c, hipMalloc(&en.d_emb, sizeof(double) * E.size()));
  HIPCHK(c, hipMemcpy(en.d_emb, E.data(), sizeof(double) * E.size(), hipMemcpyHostToDevice));
  const std::vector<float> E32(E.begin(), E.end());
  HIPCHK(c, hipMalloc(&en.d_emb32, sizeof(float) * E32.size()));
  HIPCHK(c, hipMemcpy(en.d_emb32, E32.data(), sizeof(float) * E32.size(), hipMemcpyHostToDevice));
  return DP_OK;
}

int upload_model(dp_ctx *c) {
  const HostModel &m = c->hm;
  Dims &d = c->dims;
  d = Dims{};
  d.ntypes = (int)m.ntypes;
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
  for (int l = 0; l <= d.n_fit + 1; ++l) d.fw[l] = (int)m.fit_w[l];
  if (d.M2 < 1 || d.M2 > 16 || d.M2 > d.M1) return fail(c, DP_E_MODEL, "M2 must be 1..16 and <= M1");
  if (!(d.rcut > 0 && d.rcut < 42.9)) return fail(c, DP_E_MODEL, "rcut must lie in (0, 42.9) A");
  if (!(d.rcut_smth >= 0 && d.rcut_smth < d.rcut)) return fail(c, DP_E_MODEL, "need 0 <= rcut_smth < rcut");
  if (!(m.desc_norm > 0)) return fail(c, DP_E_MODEL, "desc_norm must be positive");
  if (d.nnei < 1) return fail(c, DP_E_MODEL, "sum of sel must be positive");
  // embedding dims are kept in c->dims too (the teacher's)
  {
    Dims e;
    int rc = emb_dims(c, m, e);
    if (rc) return rc;
    d = e;
  }
  int rc = upload_emb(c, m, c->en[0]);
  if (rc) return rc;
  c->en[0].ready = true;
  const int T = d.ntypes;
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
  if (c->d_fit) (void)hipFree(c->d_fit);
  if (c->d_fit32) (void)hipFree(c->d_fit32);
  c->d_fit = nullptr;
  c->d_fit32 = nullptr;
  HIPCHK(c, hipMalloc(&c->d_fit, sizeof(double) * F.size()));
  HIPCHK(c, hipMemcpy(c->d_fit, F.data(), sizeof(double) * F.size(), hipMemcpyHostToDevice));
  const std::vector<float> F32(F.begin(), F.end());
  HIPCHK(c, hipMalloc(&c->d_fit32, sizeof(float) * F32.size()));
  HIPCHK(c, hipMemcpy(c->d_fit32, F32.data(), sizeof(float) * F32.size(), hipMemcpyHostToDevice));
  return DP_OK;
}

// Mixed-precision weights: per (t,u) the LDS image of the embedding net, and
// the fused fitting net's operand images (16-bit, lane by lane).
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

// Mixed-precision LDS images of the embedding nets of m into en.
int upload_emb_mix(dp_ctx *c, const HostModel &m, EmbNets &en) {
  en.tab_ok = false;  // the table follows the weights and the precision
  const Dims &d = en.d;
  const int prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  const int shape = mix_shape_id(d);
  if (en.d_wide) (void)hipFree(en.d_wide);
  en.d_wide = nullptr;
  en.wide = false;
  if (shape < 0) {
    // nets wider than the register-resident kernels: the GEMM path
    const char *why = nullptr;
    if (!wide_supported(d, &why))
      return fail(c, DP_E_MODEL,
                  std::string("mixed precision takes embedding widths 25-50-100 and 16-32-100 (register-resident) "
                              "or wide nets: ") + why);
    const int T = d.ntypes;
    std::vector<unsigned char> buf;
    for (int t = 0; t < T; ++t)
      for (int u = 0; u < T; ++u) {
        const double *W[MAXL], *b[MAXL];
        for (int l = 0; l < d.n_emb; ++l) {
          W[l] = m.eW[m.eidx(t, u, l)].data();
          b[l] = m.eb[m.eidx(t, u, l)].data();
        }
        wide_pack_net(d, W, b, prec, buf, en.wnet[t * T + u]);
      }
    HIPCHK(c, hipMalloc(&en.d_wide, buf.size()));
    HIPCHK(c, hipMemcpy(en.d_wide, buf.data(), buf.size(), hipMemcpyHostToDevice));
    en.wide = true;
    en.mix_shape = -1;
    return DP_OK;
  }
  if (mix_lds_bytes(shape, d.ntypes, 2) > 163840 || mix_lds_bytes(shape, d.ntypes, 1) > 163840)
    return fail(c, DP_E_MODEL, "too many atom types for the mixed-precision LDS layout");
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
  if (en.d_mix) (void)hipFree(en.d_mix);
  en.d_mix = nullptr;
  HIPCHK(c, hipMalloc(&en.d_mix, nets.size()));
  HIPCHK(c, hipMemcpy(en.d_mix, nets.data(), nets.size(), hipMemcpyHostToDevice));
  en.mix_shape = shape;
  return DP_OK;
}

int upload_mix(dp_ctx *c) {
  const HostModel &m = c->hm;
  const Dims &d = c->dims;
  const int prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  // layers below n16 hold 16-bit weights, the later hidden layers hi + lo pairs
  const int n16 = std::min(2, d.n_fit);
  const char *why = nullptr;
  if (!fit_mix_supported(d, &why)) return fail(c, DP_E_MODEL, why);
  int rc = upload_emb_mix(c, m, c->en[0]);
  if (rc) return rc;
  if (c->en[1].ready) {
    rc = upload_emb_mix(c, c->shm, c->en[1]);
    if (rc) return rc;
  }
  const int T = d.ntypes;
  std::vector<const double *> Wp, bp;
  for (int t = 0; t < T; ++t)
    for (int l = 0; l <= d.n_fit; ++l) {
      Wp.push_back(m.fW[m.fidx(t, l)].data());
      bp.push_back(m.fb[m.fidx(t, l)].data());
    }
  std::vector<unsigned char> F;
  FitMixOffsets fo{};
  fit_mix_pack(d, prec, n16, Wp.data(), bp.data(), F, fo);
  if (c->d_fit_mix) (void)hipFree(c->d_fit_mix);
  c->d_fit_mix = nullptr;
  HIPCHK(c, hipMalloc(&c->d_fit_mix, F.size()));
  HIPCHK(c, hipMemcpy(c->d_fit_mix, F.data(), F.size(), hipMemcpyHostToDevice));
  c->fmo = fo;
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

constexpr int NMARK = 10;
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
  const EmbNets &en = c->en[c->active];
  EmbedArgs ea{};
  ea.d = en.d;
  ea.eo = en.eo;
  ea.ew = en.d_emb;
  ea.atom_of_pos = c->ov_atom_of_pos ? c->ov_atom_of_pos : w.atom_of_pos;
  ea.pos_of_atom = w.pos_of_atom;
  ea.type_start = c->ov_type_start ? c->ov_type_start : w.type_start;
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

// DP_MIX_FP32: the same buffers read as float, the FP32 weight copies
EmbedArgs32 embed_args32(dp_ctx *c, int64_t n, int64_t rows, double *F) {
  const EmbedArgs e = embed_args(c, n, rows, F);
  EmbedArgs32 a{};
  a.d = e.d;
  a.eo = e.eo;
  a.ew = c->en[c->active].d_emb32;
  a.atom_of_pos = e.atom_of_pos;
  a.pos_of_atom = e.pos_of_atom;
  a.type_start = e.type_start;
  a.rows = e.rows;
  a.natoms = e.natoms;
  a.xw = e.xw;
  a.nlist = e.nlist;
  a.nreal = e.nreal;
  a.rt = c->ws.rt32;
  a.dr = e.dr;
  a.T = (float *)e.T;
  a.D = (float *)e.D;
  a.dD = (const float *)e.dD;
  a.force = e.force;
  a.vir_part = e.vir_part;
  a.net_deriv = e.net_deriv;
  return a;
}

FitArgs fit_args(dp_ctx *c, int64_t rows) {
  Workspace &w = c->ws;
  FitArgs fa{};
  fa.d = c->dims;
  fa.fo = c->fo;
  fa.fwt = c->d_fit;
  fa.type_start = c->ov_type_start ? c->ov_type_start : w.type_start;
  fa.atom_of_pos = c->ov_atom_of_pos ? c->ov_atom_of_pos : w.atom_of_pos;
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

FitArgs32 fit_args32(dp_ctx *c, int64_t rows) {
  const FitArgs f = fit_args(c, rows);
  FitArgs32 a{};
  a.d = f.d;
  a.fo = f.fo;
  a.fwt = c->d_fit32;
  a.type_start = f.type_start;
  a.atom_of_pos = f.atom_of_pos;
  a.rows = f.rows;
  a.X0 = (float *)f.X0;
  for (int l = 0; l <= MAXF; ++l) {
    a.Y[l] = (float *)f.Y[l];
    a.Tt[l] = (float *)f.Tt[l];
    a.G[l] = (float *)f.G[l];
  }
  a.eatom = f.eatom;
  return a;
}

MixArgs mix_args(dp_ctx *c, int64_t rows, double *F) {
  Workspace &w = c->ws;
  const EmbNets &en = c->en[c->active];
  MixArgs ma{};
  ma.d = en.d;
  ma.shape = en.mix_shape;
  ma.prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  ma.nets = en.d_mix;
  ma.rows = rows;
  ma.atom_of_pos = c->ov_atom_of_pos ? c->ov_atom_of_pos : w.atom_of_pos;
  ma.xw = w.xw;
  ma.nlist = w.nlist;
  ma.nreal = w.nreal;
  ma.rt = w.rt32;
  for (int k = 0; k < 3; ++k) ma.L[k] = c->box_L[k];
  ma.T32 = w.T32;
  ma.dT32 = w.dT32;
  ma.force = F;
  ma.vir_part = w.vir_part;
  ma.net_deriv = c->keep ? w.net_deriv : nullptr;
  ma.tab = nullptr;
  if (c->active == 1 && c->use_tab && en.tab_ok) {
    ma.tab = en.d_tab;
    ma.tab_inv_ds = (float)(TAB_K / en.tab_shi);
    ma.tab_shi = (float)en.tab_shi;
    ma.pimg = (const unsigned char *)en.d_tab + (size_t)c->dims.ntypes * c->dims.ntypes * TAB_BYTES;
    ma.defer = w.defer;
    ma.defer_count = &w.status->defer_count;
  }
  return ma;
}

FitMixArgs fitmix_args(dp_ctx *c, int64_t rows) {
  Workspace &w = c->ws;
  FitMixArgs fa{};
  fa.d = c->dims;
  fa.fo = c->fmo;
  fa.w = c->d_fit_mix;
  fa.prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  fa.nsplit = c->n16;
  fa.type_start = c->ov_type_start ? c->ov_type_start : w.type_start;
  fa.atom_of_pos = c->ov_atom_of_pos ? c->ov_atom_of_pos : w.atom_of_pos;
  fa.rows = rows;
  fa.T32 = w.T32;
  fa.tbuf = w.tbuf;
  fa.dT32 = w.dT32;
  fa.eatom = w.eatom;
  fa.inv_nc = (float)c->dims.inv_nc;
  return fa;
}

int64_t eval_rows(const dp_ctx *c, int64_t n) {
  if (c->ov_atom_of_pos) return c->ov_rows;
  return (n + ROW_TILE - 1) / ROW_TILE * ROW_TILE + (int64_t)ROW_TILE * c->dims.ntypes;
}

// Formatted neighbour list and environment matrix of the current frame.
void eval_lists(dp_ctx *c, int64_t n, const double L[3]) {
  Workspace &w = c->ws;
  for (int k = 0; k < 3; ++k) c->box_L[k] = L[k];
  const Dims &d = c->dims;
  hipStream_t s = c->stream;
  // the mixed path's FP32 environment rows come out of the format kernel
  // (it has each slot's neighbour and position at hand); the FP64 path's
  // rows and displacements from the environment kernel
  const bool fused = w.rt32 && !w.dr;
  tmark(c, 1);
  launch_format(s, n, w.xw, d, L, w.cand, w.cand_n, w.cand_cap, w.nlist, w.nreal, &w.status->overflow,
                w.status->max_real, &w.status->flags, fused ? w.rt32 : nullptr);
  tmark(c, 2);
  if (!fused) launch_env(s, n, w.xw, d, L, w.nlist, w.nreal, w.rt, w.rt32, w.dr);
  tmark(c, 3);
}

// Table of the active student nets (mixed precision): built on the first
// evaluation after the nets or the precision change, over s in
// [0, 1.25 x the largest s of that frame]; tiles with a larger s evaluate the
// layers instead.
int ensure_table(dp_ctx *c, int64_t n) {
  EmbNets &en = c->en[c->active];
  if (c->active != 1 || !c->use_tab || !prec16(c->precision) || en.tab_ok || n <= 0) return DP_OK;
  if (!mix_tab_fits(en.mix_shape, c->dims.ntypes)) return DP_OK;
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  launch_fill_u32(s, &w.status->smax_bits, 1, 0u);
  launch_smax(s, n, c->dims, w.nreal, w.rt32, &w.status->smax_bits);
  uint32_t bits = 0;
  HIPCHK(c, hipMemcpyAsync(&bits, &w.status->smax_bits, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  float smax;
  std::memcpy(&smax, &bits, 4);
  const double shi = smax > 0.f ? 1.25 * (double)smax : 1.0;
  if (!en.d_tab) {
    if (c->noalloc) return DP_OK;  // no table yet and no allocation allowed: the layers are evaluated
    HIPCHK(c, hipMalloc(&en.d_tab, (size_t)c->dims.ntypes * c->dims.ntypes * (TAB_BYTES + PIMG_BYTES)));
  }
  const int nets = c->dims.ntypes * c->dims.ntypes, prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  launch_student_table(s, en.d, en.eo, en.d_emb, prec, shi, en.d_tab);
  launch_student_pimg(s, nets, en.d_tab, prec, (unsigned char *)en.d_tab + (size_t)nets * TAB_BYTES);
  HIPCHK(c, hipGetLastError());
  en.tab_shi = shi;
  en.tab_ok = true;
  return DP_OK;
}

// Arguments of the wide-path kernels (buffers as laid out by wide_forward).
WideArgs wide_args(dp_ctx *c, int64_t n) {
  Workspace &w = c->ws;
  const EmbNets &en = c->en[c->active];
  WideArgs a{};
  a.d = en.d;
  a.prec = c->precision == DP_MIX_FP16 ? 0 : 1;
  a.split = c->wb.split;
  a.n = n;
  a.xw = w.xw;
  a.nlist = w.nlist;
  a.nreal = w.nreal;
  a.rt = w.rt32;
  for (int k = 0; k < 3; ++k) a.L[k] = c->box_L[k];
  a.poff = c->wb.poff;
  a.cnt = c->wb.cnt;
  const int nets = en.d.ntypes * en.d.ntypes;
  for (int k = 0; k < nets; ++k) {
    a.row0[k] = c->wb.row0[k];
    a.w0[k] = (const float *)(en.d_wide + en.wnet[k].w[0]);
    a.b0[k] = (const float *)(en.d_wide + en.wnet[k].b[0]);
  }
  a.X0 = c->wb.X[0];
  a.G = c->wb.X[c->wb.out];
  a.T32 = w.T32;
  a.dT32 = w.dT32;
  a.vir_part = w.vir_part;
  a.net_deriv = c->keep ? w.net_deriv : nullptr;
  return a;
}

// Wide embedding nets, forward: pair counts (one host read-back: the
// activation rows are laid out per net from them), layer 0, the GEMM layers
// (value and tangent rows), T.  Buffers grow by 1/4 beyond the need.
int wide_forward(dp_ctx *c, int64_t n) {
  auto &wb = c->wb;
  const EmbNets &en = c->en[c->active];
  const Dims &d = en.d;
  hipStream_t s = c->stream;
  const int T = d.ntypes, nets = T * T;
  wb.ok = false;
  wb.split = c->wide_split;
  if (n > wb.n_cap) {
    if (wb.poff) (void)hipFree(wb.poff);
    wb.poff = wb.cnt = nullptr;
    wb.n_cap = 0;
    const int64_t cap = n + n / 4;
    if (hipMalloc(&wb.poff, sizeof(int32_t) * ((size_t)cap * T + WIDE_NETS)) != hipSuccess)
      return fail(c, DP_E_OOM, "wide embedding: out of device memory (pair offsets)");
    wb.cnt = wb.poff + (size_t)cap * T;
    wb.n_cap = cap;
  }
  launch_fill_u32(s, (uint32_t *)wb.cnt, nets, 0u);
  WideArgs a = wide_args(c, n);
  launch_wide_count(s, a);
  HIPCHK(c, hipMemcpyAsync(wb.cnt_h, wb.cnt, sizeof(int32_t) * nets, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  wb.row0[0] = 0;
  for (int k = 0; k < nets; ++k)
    wb.row0[k + 1] = wb.row0[k] + (2 * (int64_t)wb.cnt_h[k] + WIDE_ROWPAD - 1) / WIDE_ROWPAD * WIDE_ROWPAD;
  int maxw = 0;
  for (int l = 1; l <= d.n_emb; ++l) maxw = std::max(maxw, d.ew[l]);
  const size_t need = (size_t)wb.row0[nets] * maxw * (1 + wb.split);
  if (need > wb.x_cap) {
    for (auto &x : wb.X) {
      if (x) (void)hipFree(x);
      x = nullptr;
    }
    wb.x_cap = 0;
    const size_t cap = need + need / 4;
    if (hipMalloc(&wb.X[0], 2 * cap) != hipSuccess || hipMalloc(&wb.X[1], 2 * cap) != hipSuccess)
      return fail(c, DP_E_OOM, "wide embedding: out of device memory (activations)");
    wb.x_cap = cap;
  }
  wb.out = 0;
  a = wide_args(c, n);
  launch_wide_l0(s, a);
  int cur = 0;
  for (int l = 1; l < d.n_emb; ++l) {
    const int Kb = d.ew[l], N = d.ew[l + 1], sp = wb.split;
    for (int k = 0; k < nets; ++k) {
      if (wb.cnt_h[k] == 0) continue;
      WideGemm g{};
      g.A = wb.X[cur] + wb.row0[k] * (Kb << sp);
      g.Bt = (const uint16_t *)(en.d_wide + en.wnet[k].w[l]);
      g.bias = (const float *)(en.d_wide + en.wnet[k].b[l]);
      g.Y = wb.X[cur ^ 1] + wb.row0[k] * (N << sp);
      g.rows = wb.row0[k + 1] - wb.row0[k];
      g.K = Kb << sp;
      g.Kb = Kb;
      g.N = N;
      g.split = sp;
      g.skip = N == Kb ? 1 : (N == 2 * Kb ? 2 : 0);
      launch_wide_gemm(s, g, a.prec);
    }
    cur ^= 1;
  }
  wb.out = cur;
  a = wide_args(c, n);
  launch_wide_T(s, a);
  wb.ok = true;
  return DP_OK;
}

// Networks of the forward half with the active embedding set: embedding +
// descriptor, fitting net forward, energy into E.
void eval_nets_fwd(dp_ctx *c, int64_t n, double *E) {
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  const int64_t rows = eval_rows(c, n);
  if (c->precision == DP_FP64) {
    launch_embed_fwd_f64(s, embed_args(c, n, rows, nullptr));
    tmark(c, 4);
    launch_fit_f64(s, fit_args(c, rows), 1);
    tmark(c, 8);
  } else if (c->precision == DP_MIX_FP32) {
    launch_embed_fwd_f32(s, embed_args32(c, n, rows, nullptr));
    tmark(c, 4);
    launch_fit_f32(s, fit_args32(c, rows), 1);
    tmark(c, 8);
  } else {
    (void)ensure_table(c, n);  // a failed table build leaves tab_ok false: the layers are evaluated
    if (c->en[c->active].wide) {
      const int rc = wide_forward(c, n);
      if (rc) c->pending_rc = rc;
      c->stats.wide_evals += 1;
    } else {
      const MixArgs ma = mix_args(c, rows, nullptr);
      if (ma.tab) c->stats.table_evals += 1;
      launch_embed_mix(s, ma, 1, mix_grid(rows));
    }
    tmark(c, 4);
    launch_fit_mix(s, fitmix_args(c, rows), 1);
    tmark(c, 8);
  }
  launch_sum(s, w.eatom, n, w.partial, E, 1.0);
  if (c->active == 1) c->stats.student_evals += 1;
}

// Forward half of an evaluation.  Leaves everything the backward half
// needs in the workspace.
void eval_forward(dp_ctx *c, int64_t n, const double L[3]) {
  eval_lists(c, n, L);
  eval_nets_fwd(c, n, c->ws.energy);
}

// Whether the mixed backward of this evaluation can scatter the pair forces
// cell by cell (full evaluation, cell list of these lists with 3..255 cells
// per axis, an affine-last-layer net set whose kernel fits the LDS); fills
// the kernel arguments.
bool cell_scatter_args(dp_ctx *c, int64_t n, const MixArgs &ma, CellArgs &ca, int &threads, size_t &lds) {
  Workspace &w = c->ws;
  if (c->scatter != 0 || c->ov_atom_of_pos || c->n_force > 0 || !c->cgrid_ok || !w.cell_part || n <= 0) return false;
  for (int a = 0; a < 3; ++a)
    if (c->cgrid.nc[a] < 3 || c->cgrid.nc[a] > 255) return false;
  // atoms per cell kept in the LDS accumulator (atoms beyond it add their
  // forces with global atomics): up to twice the mean occupancy plus slack,
  // at most CELL_CAP, and at least the mean plus 16; within that range the
  // kernel takes the most waves the LDS allows
  const int64_t ncell = (int64_t)c->cgrid.nc[0] * c->cgrid.nc[1] * c->cgrid.nc[2];
  const int64_t mean = (n + ncell - 1) / ncell;
  const int want = (int)std::max<int64_t>(32, std::min<int64_t>(CELL_CAP, (2 * mean + 16 + 15) / 16 * 16));
  const int need = (int)std::min<int64_t>(want, std::max<int64_t>(16, mean + 16));
  int cap = 0;
  if (!embed_cells_config(ma, want, need, &cap, &threads, &lds)) return false;
  ca.cell_start = w.cell_start;
  ca.cell_atoms = w.cell_atoms;
  ca.cell_of = w.cell_of;
  ca.code = w.cell_code;
  for (int a = 0; a < 3; ++a) ca.nc[a] = c->cgrid.nc[a];
  ca.cap = cap;
  ca.ncell = ncell;
  ca.n = n;
  ca.part = w.cell_part;
  return true;
}

// Backward half (the adjoint): fitting net backward to dE/dD, then the
// embedding backward with the force scatter into F and the virial into V.
void eval_backward(dp_ctx *c, int64_t n, double *F, double *V) {
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  const int64_t rows = eval_rows(c, n);
  if (!prec16(c->precision)) {
    const bool f32 = c->precision == DP_MIX_FP32;
    if (f32) launch_fit_f32(s, fit_args32(c, rows), 2);
    else launch_fit_f64(s, fit_args(c, rows), 2);
    tmark(c, 5);
    launch_zero(s, F, 3 * (c->n_force > 0 ? c->n_force : n));
    const int grid = embed_bwd_grid(rows);
    tmark(c, 6);
    if (f32) launch_embed_bwd_f32(s, embed_args32(c, n, rows, F), grid);
    else launch_embed_bwd_f64(s, embed_args(c, n, rows, F), grid);
    tmark(c, 9);
    tmark(c, 7);
    launch_sum9(s, w.vir_part, grid, V);
  } else {
    launch_fit_mix(s, fitmix_args(c, rows), 2);
    tmark(c, 5);
    launch_zero(s, F, 3 * (c->n_force > 0 ? c->n_force : n));
    tmark(c, 6);
    if (c->en[c->active].wide) {
      if (c->wb.ok) {
        WideArgs a = wide_args(c, n);
        a.force = F;
        launch_wide_bwd(s, a);
        tmark(c, 9);
        tmark(c, 7);
        launch_sum9(s, w.vir_part, (int)std::min<int64_t>(n, WIDE_GRID), V);
      } else {
        tmark(c, 9);
        tmark(c, 7);
        launch_zero(s, V, 9);
      }
      tnext(c);
      return;
    }
    const MixArgs ma = mix_args(c, rows, F);
    CellArgs ca{};
    int threads = 0;
    size_t lds = 0;
    // with the table, nets with a neighbour beyond its range are deferred to
    // a layer pass after the main kernel; its virial partials follow the
    // main kernel's
    if (ma.tab) launch_fill_u32(s, ma.defer_count, 1, 0u);
    auto deferred = [&](int grid) {
      if (!ma.tab) return 0;
      MixArgs md = ma;
      md.vir_part = w.vir_part + (size_t)9 * grid;
      launch_embed_defer(s, md);
      return DEFER_GRID;
    };
    if (cell_scatter_args(c, n, ma, ca, threads, lds)) {
      const int grid = cells_grid(ca.ncell);
      launch_embed_cells(s, ma, ca, grid, threads, lds);
      tmark(c, 9);
      launch_cell_gather(s, ca, F);
      const int gd = deferred(grid);
      tmark(c, 7);
      launch_sum9(s, w.vir_part, grid + gd, V);
      c->stats.cell_scatter += 1;
    } else {
      const int grid = mix_grid(rows);
      launch_embed_mix(s, ma, 2, grid);
      tmark(c, 9);
      const int gd = deferred(grid);
      tmark(c, 7);
      launch_sum9(s, w.vir_part, grid + gd, V);
    }
  }
  tnext(c);
}

void eval_body(dp_ctx *c, int64_t n, const double L[3], double *F) {
  eval_forward(c, n, L);
  eval_backward(c, n, F, c->ws.virial);
}

// Student judge on the frame just evaluated (lists, environment and the
// student's forces F in place): the teacher's networks on the same frame,
// then the force RMSE into the status block (read by the next status sync).
void eval_judge(dp_ctx *c, int64_t n) {
  Workspace &w = c->ws;
  const bool tim = c->timing;
  c->timing = false;
  c->active = 0;
  eval_nets_fwd(c, n, w.energy_j);
  eval_backward(c, n, w.force_j, w.virial_j);
  c->active = 1;
  c->timing = tim;
}

void build_lists(dp_ctx *c, int64_t n, const CellGrid &g, double rlist, const uint32_t *cond) {
  Workspace &w = c->ws;
  launch_cells(c->stream, n, w.xw, g, w.cell_of, w.cell_start, w.cell_fill, w.cell_atoms, w.cell_code, w.scan_tmp,
               cond);
  c->cgrid = g;
  c->cgrid_ok = true;
  launch_candidates(c->stream, n, w.xw, g, w.cell_start, w.cell_atoms, rlist, w.cand_cap, w.cand, w.cand_n,
                    &w.status->flags, cond);
}

int read_status(dp_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->h_status, c->ws.status, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->pending_rc != DP_OK) {
    const int rc = c->pending_rc;
    c->pending_rc = DP_OK;
    return rc;
  }
  c->stats.sel_overflow = (int64_t)c->h_status->overflow;
  for (int t = 0; t < MAXT; ++t) c->stats.max_real[t] = c->h_status->max_real[t];
  c->stats.nlist_builds = (int64_t)c->h_status->nbuild;
  return DP_OK;
}

// Judge the student's forces F of the frame just evaluated against the
// teacher's; on a rejection take the teacher's forces, energy and virial for
// this frame and switch the context to the teacher.  With judge_side > 0
// the teacher is evaluated only on a cube of that side placed by SplitMix64
// from the step number (stream 0x6a75646765, counters 3 step + axis) and on
// the atoms within rc of it, which gives the cube's atoms their exact teacher
// forces; the RMSE is taken over the cube.  A rejected sample is confirmed
// by a full teacher evaluation before the fallback.
int judge_step(dp_ctx *c, int64_t n, double *F, int64_t step, const double L[3]) {
  Workspace &w = c->ws;
  hipStream_t s = c->stream;
  const double rc = c->dims.rcut;
  const double side = c->judge_side;
  if (side > 0.0 && side + 2.0 * rc < std::min(L[0], std::min(L[1], L[2]))) {
    double ctr[3];
    for (int a = 0; a < 3; ++a)
      ctr[a] = L[a] * ((double)(sm64(0x6a75646765ull, 3ull * (uint64_t)step + (uint64_t)a) >> 11) * 0x1.0p-53);
    launch_judge_mark(s, n, w.xw, ctr, L, 0.5 * side, 0.5 * side + rc, w.judge_mark);
    launch_type_sort(s, n, w.xw, c->dims.ntypes, w.sub_blk, w.sub_type_count, w.sub_type_start, nullptr,
                     w.sub_atom_of_pos, w.rows_cap, w.judge_mark);
    launch_copy_i32(s, w.sub_type_start + c->dims.ntypes, &w.status->sub_rows);
    int rc2 = read_status(c);
    if (rc2) return rc2;
    c->ov_atom_of_pos = w.sub_atom_of_pos;
    c->ov_type_start = w.sub_type_start;
    c->ov_rows = c->h_status->sub_rows;
    eval_judge(c, n);
    c->ov_atom_of_pos = c->ov_type_start = nullptr;
    c->ov_rows = 0;
    launch_force_rmse_masked(s, F, w.force_j, n, w.judge_mark, w.rmse_part, &w.status->judge_rmse,
                             &w.status->judge_count);
    HIPCHK(c, hipGetLastError());
    rc2 = read_status(c);
    if (rc2) return rc2;
    if (c->h_status->flags & FLAG_HALT) return DP_OK;  // forces of a stopped step: the caller handles the flag
    c->stats.last_judge_rmse = c->h_status->judge_rmse;
    c->stats.judge_atoms = (int64_t)c->h_status->judge_count;
    if (c->h_status->judge_rmse <= c->judge_max) return DP_OK;
  }
  eval_judge(c, n);
  launch_force_rmse(s, F, w.force_j, n, w.rmse_part, &w.status->judge_rmse);
  HIPCHK(c, hipGetLastError());
  int rc3 = read_status(c);
  if (rc3) return rc3;
  if (c->h_status->flags & FLAG_HALT) return DP_OK;
  const double r = c->h_status->judge_rmse;
  c->stats.last_judge_rmse = r;
  c->stats.judge_atoms = n;
  if (!(r <= c->judge_max)) {  // a NaN rejects as well
    HIPCHK(c, hipMemcpyAsync(F, w.force_j, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w.energy, w.energy_j, sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w.virial, w.virial_j, sizeof(double) * 9, hipMemcpyDeviceToDevice, s));
    c->active = 0;
    c->stats.teacher_fallbacks += 1;
  }
  return DP_OK;
}

__global__ void k_reset_status(DevStatus *st, uint32_t flags) {
  if (threadIdx.x == 0) {
    st->flags = flags;
    st->fault_step = -1;
    st->overflow = 0;
    for (int t = 0; t < MAXT; ++t) st->max_real[t] = 0;
  }
}

// ---------------------------------------------------------------------------
// student helpers
// ---------------------------------------------------------------------------
constexpr int64_t ST_Q_LS = 1ll << 36;     // first sample index of the refit
constexpr int64_t ST_Q_CHECK = 1ll << 37;  // first sample index of the held-out check
constexpr int64_t ST_CHECK_N = 4096;
constexpr int64_t ST_DRAW_MAX = 64;         // batches drawn (samples + teacher targets) per launch, at most
constexpr int64_t ST_DRAW_SAMPLES = 262144; // and at most this many samples per net

// samples per net one draw holds for batches of `batch`
int64_t draw_capacity(int64_t batch) {
  return std::max<int64_t>(ST_CHECK_N, std::max<int64_t>(batch, std::min<int64_t>(batch * ST_DRAW_MAX, ST_DRAW_SAMPLES)));
}

int ensure_student(dp_ctx *c, int64_t batch) {
  const int nets = c->dims.ntypes * c->dims.ntypes;
  const int M1 = c->dims.M1;
  const StudentLayout L = student_layout(M1);
  Student *st = c->st;
  if (st && st->cap >= batch && st->cap_draw >= draw_capacity(batch) && st->nets == nets && st->M1 == M1)
    return DP_OK;
  std::vector<float> keep;
  bool had = false;
  int64_t t = 0;
  if (st && st->have_params && st->nets == nets && st->M1 == M1) {
    keep.resize((size_t)nets * L.np);
    HIPCHK(c, hipMemcpy(keep.data(), st->params, sizeof(float) * keep.size(), hipMemcpyDeviceToHost));
    had = true;
    t = st->t;
  }
  free_student(c);
  st = new Student();
  c->st = st;
  st->nets = nets;
  st->M1 = M1;
  st->np = L.np;
  st->cap = std::max<int64_t>(batch, ST_CHECK_N);
  st->cap_draw = draw_capacity(batch);
  const int64_t cap = st->cap, capd = st->cap_draw, nblk = cap / 64, NE = (int64_t)SNF * SNF + (int64_t)SNF * M1;
  std::vector<std::pair<void **, size_t>> plan;
  auto add = [&](void **p, size_t bytes) { plan.push_back({p, bytes}); };
  add((void **)&st->params, sizeof(float) * nets * L.np);
  add((void **)&st->m, sizeof(float) * nets * L.np);
  add((void **)&st->v, sizeof(float) * nets * L.np);
  add((void **)&st->gout, sizeof(float) * nets * L.np);
  add((void **)&st->gpart, sizeof(float) * nets * nblk * L.np);
  add((void **)&st->lpart, sizeof(double) * nets * nblk * 2);
  add((void **)&st->s, sizeof(double) * nets * capd);
  add((void **)&st->wt, sizeof(float) * nets * capd);
  add((void **)&st->G, sizeof(double) * nets * capd * M1);
  add((void **)&st->lspart, sizeof(double) * nets * st_ls_blocks() * NE);
  add((void **)&st->lsfold, sizeof(double) * nets * ST_LS_FOLD * NE);
  add((void **)&st->X, sizeof(double) * nets * SNF * M1);
  add((void **)&st->chk, sizeof(double) * nets * nblk * 2);
  add((void **)&st->loss, sizeof(double) * nets);
  add((void **)&st->status, sizeof(int32_t) * nets);
  size_t off = 0;
  for (auto &pr : plan) off += (pr.second + 255) / 256 * 256;
  if (hipMalloc(&st->base, off) != hipSuccess) {
    (void)hipGetLastError();
    free_student(c);
    return fail(c, DP_E_OOM, "student buffers: allocation of " + std::to_string(off) + " bytes failed");
  }
  size_t o = 0;
  for (auto &pr : plan) {
    *pr.first = (char *)st->base + o;
    o += (pr.second + 255) / 256 * 256;
  }
  if (had) {
    HIPCHK(c, hipMemcpy(st->params, keep.data(), sizeof(float) * keep.size(), hipMemcpyHostToDevice));
    st->have_params = true;
    st->t = t;
  }
  return DP_OK;
}

bool lists_ready(const dp_ctx *c) { return c->has_model && c->ws.n_cap >= 0 && c->last_n > 0; }

// nb consecutive batches of samples (indices q0 .. q0 + nb * batch - 1 per
// net) and their teacher targets, laid out [nb][nets][batch]
void st_draw(dp_ctx *c, uint64_t seed, int64_t q0, int64_t batch, int nb = 1) {
  Workspace &w = c->ws;
  Student *st = c->st;
  StSampleArgs sa{};
  sa.d = c->dims;
  sa.type_count = w.type_count;
  sa.type_start = w.type_start;
  sa.atom_of_pos = w.atom_of_pos;
  sa.nreal = w.nreal;
  sa.xw = w.xw;
  sa.nlist = w.nlist;
  for (int k = 0; k < 3; ++k) sa.L[k] = c->box_L[k];
  sa.seed = seed;
  sa.q0 = q0;
  sa.batch = (int)batch;
  sa.nb = nb;
  sa.s = st->s;
  sa.wt = st->wt;
  launch_st_sample(c->stream, sa);
  StTeacherArgs ta{};
  ta.d = c->en[0].d;
  ta.eo = c->en[0].eo;
  ta.ew = c->en[0].d_emb;
  ta.batch = (int)batch;
  ta.nb = nb;
  ta.s = st->s;
  ta.G = st->G;
  launch_st_teacher(c->stream, ta);
}

// gradient of batch k of the last draw
void st_grad(dp_ctx *c, int64_t batch, int k = 0) {
  Student *st = c->st;
  const int64_t o = (int64_t)k * st->nets * batch;
  StGradArgs ga{};
  ga.M1 = st->M1;
  ga.nets = st->nets;
  ga.batch = (int)batch;
  ga.params = st->params;
  ga.s = st->s + o;
  ga.wt = st->wt + o;
  ga.G = st->G + o * st->M1;
  ga.gpart = st->gpart;
  ga.lpart = st->lpart;
  launch_st_grad(c->stream, ga);
}

void st_adam(dp_ctx *c, int64_t batch, const dp_student_cfg &cfg, float *g_out) {
  Student *st = c->st;
  StAdamArgs aa{};
  aa.M1 = st->M1;
  aa.nets = st->nets;
  aa.nblk = (int)(batch / 64);
  aa.params = st->params;
  aa.m = st->m;
  aa.v = st->v;
  aa.gpart = st->gpart;
  aa.lpart = st->lpart;
  aa.lr = (float)cfg.lr;
  aa.b1 = (float)cfg.beta1;
  aa.b2 = (float)cfg.beta2;
  aa.eps = (float)cfg.eps;
  const double tt = (double)(st->t + 1);
  aa.c1 = (float)(1.0 / (1.0 - std::pow(cfg.beta1, tt)));
  aa.c2 = (float)(1.0 / (1.0 - std::pow(cfg.beta2, tt)));
  aa.loss = st->loss;
  aa.g_out = g_out;
  launch_st_adam(c->stream, aa);
}

// host initialisation: W1 ~ N(0, (2/smax)^2), b1 ~ N(0,1), W2 ~ N(0, 2/48),
// b2 ~ N(0,1), W3 ~ N(0, 2/(32+M1)), b3 = 0; normal deviates by Box-Muller
// from SplitMix64 (stream seed ^ 0xa0761d6478bd642f, counters net*2^40 + k)
void st_init_params(const Student &st, uint64_t seed, const std::vector<double> &smax, std::vector<float> &P) {
  const StudentLayout L = student_layout(st.M1);
  P.assign((size_t)st.nets * L.np, 0.f);
  const uint64_t sd = seed ^ 0xa0761d6478bd642full;
  for (int net = 0; net < st.nets; ++net) {
    uint64_t k = 0;
    auto normal = [&]() {
      const uint64_t a = sm64(sd, ((uint64_t)net << 40) + k++), b = sm64(sd, ((uint64_t)net << 40) + k++);
      const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53, u2 = (double)(b >> 11) * 0x1.0p-53;
      return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    float *p = P.data() + (size_t)net * L.np;
    const double s1 = 2.0 / std::max(smax[net], 1e-3);
    for (int i = 0; i < SH1; ++i) p[L.o_w1 + i] = (float)(s1 * normal());
    for (int i = 0; i < SH1; ++i) p[L.o_b1 + i] = (float)normal();
    for (int i = 0; i < SH1 * SH2; ++i) p[L.o_w2 + i] = (float)(std::sqrt(2.0 / (SH1 + SH2)) * normal());
    for (int i = 0; i < SH2; ++i) p[L.o_b2 + i] = (float)normal();
    for (int i = 0; i < SH2 * st.M1; ++i) p[L.o_w3 + i] = (float)(std::sqrt(2.0 / (SH2 + st.M1)) * normal());
  }
}

int quant_of(const dp_ctx *c) {
  return c->precision == DP_MIX_FP16 ? 0 : (c->precision == DP_MIX_BF16 ? 1 : -1);
}

// Install student host model `m` (embedding 1-16-32-M1 affine) on the device.
int install_student(dp_ctx *c, HostModel &&m) {
  c->en[1].ready = false;
  c->fwd_ready = false;  // a pending backward would meet other nets
  c->shm = std::move(m);
  int rc = upload_emb(c, c->shm, c->en[1]);
  if (rc) return rc;
  if (prec16(c->precision)) {
    rc = upload_emb_mix(c, c->shm, c->en[1]);
    if (rc) return rc;
  }
  c->en[1].ready = true;
  return DP_OK;
}

// Serialise a host model as a DPMIBLOB (version 2 when the last embedding
// layer is affine).
std::vector<unsigned char> write_blob(const HostModel &m) {
  std::vector<unsigned char> b;
  auto put = [&](const void *p, size_t n) {
    const unsigned char *q = (const unsigned char *)p;
    b.insert(b.end(), q, q + n);
  };
  auto i64 = [&](int64_t v) { put(&v, 8); };
  auto f64 = [&](double v) { put(&v, 8); };
  put("DPMIBLOB", 8);
  i64(m.emb_lin ? 2 : 1);
  i64(m.ntypes);
  i64(m.n_emb);
  i64(m.n_fit);
  i64(m.M2);
  if (m.emb_lin) i64(1);
  f64(m.rcut);
  f64(m.rcut_smth);
  f64(m.desc_norm);
  for (auto v : m.sel) i64(v);
  for (auto v : m.emb_w) i64(v);
  for (int64_t l = 1; l <= m.n_fit; ++l) i64(m.fit_w[l]);
  for (int64_t t = 0; t < m.ntypes; ++t)
    for (int64_t u = 0; u < m.ntypes; ++u)
      for (int64_t l = 0; l < m.n_emb; ++l) {
        const auto &W = m.eW[m.eidx(t, u, l)];
        const auto &bb = m.eb[m.eidx(t, u, l)];
        put(W.data(), 8 * W.size());
        put(bb.data(), 8 * bb.size());
      }
  for (int64_t t = 0; t < m.ntypes; ++t)
    for (int64_t l = 0; l <= m.n_fit; ++l) {
      const auto &W = m.fW[m.fidx(t, l)];
      const auto &bb = m.fb[m.fidx(t, l)];
      put(W.data(), 8 * W.size());
      put(bb.data(), 8 * bb.size());
    }
  return b;
}

// The student host model from FP32 hidden-layer parameters and the FP64
// output layer X ([nets][33][M1]); W2 rounded as the kernels will hold it.
HostModel student_model(const dp_ctx *c, const std::vector<float> &P, const std::vector<double> &X, int quant) {
  HostModel m = c->hm;
  const int T = (int)m.ntypes, M1 = c->dims.M1;
  const StudentLayout L = student_layout(M1);
  m.n_emb = 3;
  m.emb_lin = 1;
  m.emb_w = {1, SH1, SH2, M1};
  m.eW.assign((size_t)T * T * 3, {});
  m.eb.assign((size_t)T * T * 3, {});
  for (int t = 0; t < T; ++t)
    for (int u = 0; u < T; ++u) {
      const int net = t * T + u;
      const float *p = P.data() + (size_t)net * L.np;
      const double *x = X.data() + (size_t)net * SNF * M1;
      auto &W1 = m.eW[m.eidx(t, u, 0)], &b1 = m.eb[m.eidx(t, u, 0)];
      auto &W2 = m.eW[m.eidx(t, u, 1)], &b2 = m.eb[m.eidx(t, u, 1)];
      auto &W3 = m.eW[m.eidx(t, u, 2)], &b3 = m.eb[m.eidx(t, u, 2)];
      for (int i = 0; i < SH1; ++i) {
        W1.push_back(p[L.o_w1 + i]);
        b1.push_back(p[L.o_b1 + i]);
      }
      for (int i = 0; i < SH1 * SH2; ++i) W2.push_back(st_round16(p[L.o_w2 + i], quant));
      for (int j = 0; j < SH2; ++j) b2.push_back(p[L.o_b2 + j]);
      for (int k = 0; k < SH2 * M1; ++k) W3.push_back(x[k]);
      for (int o = 0; o < M1; ++o) b3.push_back(x[SH2 * M1 + o]);
    }
  return m;
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
  c->scratch = scratch_address(device, &c->scratch_rc);
  *out = c;
  return DP_OK;
}

void dp_destroy(dp_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_ws(c->ws);
  for (auto &en : c->en) {
    if (en.d_emb) (void)hipFree(en.d_emb);
    if (en.d_emb32) (void)hipFree(en.d_emb32);
    if (en.d_mix) (void)hipFree(en.d_mix);
    if (en.d_tab) (void)hipFree(en.d_tab);
    if (en.d_wide) (void)hipFree(en.d_wide);
  }
  free_wide(c);
  free_student(c);
  if (c->d_fit) (void)hipFree(c->d_fit);
  if (c->d_fit32) (void)hipFree(c->d_fit32);
  if (c->d_fit_mix) (void)hipFree(c->d_fit_mix);
  if (c->h_status) (void)hipHostFree(c->h_status);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char *dp_last_error(const dp_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

int dp_set_model(dp_ctx *c, const void *blob, size_t nbytes, int precision) {
  if (!c || !blob) return fail(c, DP_E_ARG, "NULL argument");
  if (!prec_ok(precision)) return fail(c, DP_E_ARG, "unsupported precision policy");
  HIPCHK(c, hipSetDevice(c->device));
  c->fwd_ready = false;  // the workspace a pending backward needs is freed below
  HostModel m;
  std::string err;
  if (!parse_blob(blob, nbytes, m, err)) return fail(c, DP_E_MODEL, err);
  c->hm = std::move(m);
  free_ws(c->ws);
  c->ws_na = Workspace{};  // laid out on the static scratch: nothing to free
  free_wide(c);
  c->has_model = false;
  c->active = 0;
  c->en[1].ready = false;
  if (c->st) c->st->have_params = false;
  int rc = upload_model(c);
  if (rc) return rc;
  const char *why = nullptr;
  if (!prec16(precision) && !f64_emb_ok(c->dims, &why)) return fail(c, DP_E_MODEL, why);
  c->precision = precision;
  if (prec16(precision)) {
    rc = upload_mix(c);
    if (rc) return rc;
  }
  c->has_model = true;
  return DP_OK;
}

int dp_set_precision(dp_ctx *c, int precision) {
  if (!c) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "no model");
  if (!prec_ok(precision)) return fail(c, DP_E_ARG, "unsupported precision policy");
  const char *why = nullptr;
  if (!prec16(precision) && !f64_emb_ok(c->dims, &why)) return fail(c, DP_E_MODEL, why);
  const int old = c->precision;
  c->fwd_ready = false;  // the forward's buffers belong to the old precision
  c->precision = precision;
  if (prec16(precision)) {
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
  if ((keep != 0) != c->keep) c->fwd_ready = false;  // the backward's outputs changed
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
  // marks: 0 start, 1 lists built, 2 format, 3 env, 4 embed_fwd, 8 fitting
  // net forward kernel, 5 fitting net (energy sum, backward kernel), 6 force
  // clear, 9 embedding backward kernel, 7 embed_bwd done (gather of the
  // cell-ordered scatter)
  static const char *names[] = {"lists", "format", "env", "embed_fwd", "fit", "embed_bwd", "total",
                                "fit_fwd", "fit_bwd", "embed_bwd_main"};
  static const int from[] = {0, 1, 2, 3, 4, 6, 0, 4, 8, 6};
  static const int to[] = {1, 2, 3, 4, 5, 7, 7, 8, 5, 9};
  if (c->nev == 0) return fail(c, DP_E_ARG, "no timed evaluation");
  for (int k = 0; k < 10; ++k)
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
      if (backward) eval_backward(c, n, F, w.virial);
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
    if (fl & FLAG_KEY_CAP) return fail(c, DP_E_CAP, "more than 512 neighbours within rcut of one atom");
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

// out[idx[k]] += in[k] (three components), FP64 atomics
__global__ void k_scatter_add3(int64_t n, const int32_t *idx, const double *in, double *out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  const int32_t j = idx[k / 3];
  if (j >= 0) atomicAdd(out + 3 * (int64_t)j + k % 3, in[k]);
}

// Evaluation of the atoms [0, n_local) of a spatial brick as centres, with
// the ghost atoms [n_local, n) as neighbours only (a rank's share of the
// spatial decomposition of Section V-D).
static int compute_local_impl(dp_ctx *c, int64_t n_local, int64_t n, const double *coords, const int32_t *types,
                              const double *box, double *energy, double *forces, double *virial) {
  if (!c) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "evaluation before dp_set_model");
  if (n < 0 || n >= (1 << 26) || n_local < 0 || n_local > n) return fail(c, DP_E_ARG, "need 0 <= n_local <= natoms < 2^26");
  if (n > 0 && (!coords || !types)) return fail(c, DP_E_ARG, "NULL coords or types");
  if (c->en[c->active].wide) return fail(c, DP_E_MODEL, "local evaluation does not cover wide embedding nets");
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
  c->last_n = 0;  // the lists below cover the centres only
  for (int attempt = 0; attempt < 4; ++attempt) {
    rc = ensure_ws(c, std::max<int64_t>(n, 1), ncell, cap);
    if (rc) return rc;
    Workspace &w = c->ws;
    double *F = forces ? forces : w.force_tmp;
    tmark(c, 0);
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, w.status, 0u);
    if (n_local > 0) {
      launch_wrap(s, n, coords, types, d.ntypes, L, w.xw, &w.status->flags);
      // rows (the fitting net's and the embedding kernels') for the centres only
      launch_type_sort(s, n_local, w.xw, d.ntypes, w.blk_counts, w.type_count, w.type_start, w.pos_of_atom,
                       w.atom_of_pos, w.rows_cap);
      // the cell list holds every atom, candidate lists the centres
      launch_cells(s, n, w.xw, g, w.cell_of, w.cell_start, w.cell_fill, w.cell_atoms, w.cell_code, w.scan_tmp,
                   nullptr);
      c->cgrid = g;
      c->cgrid_ok = true;
      launch_candidates(s, n_local, w.xw, g, w.cell_start, w.cell_atoms, rlist, w.cand_cap, w.cand, w.cand_n,
                        &w.status->flags, nullptr);
      c->n_force = n;
      eval_forward(c, n_local, L);
      eval_backward(c, n_local, F, w.virial);
      c->n_force = 0;
    } else {
      if (n > 0 && forces) launch_zero(s, F, 3 * n);
      launch_zero(s, w.energy, 1);
      launch_zero(s, w.virial, 9);
      for (int k = 1; k < NMARK; ++k) tmark(c, k);
      tnext(c);
    }
    if (energy) HIPCHK(c, hipMemcpyAsync(energy, w.energy, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (virial) HIPCHK(c, hipMemcpyAsync(virial, w.virial, 9 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipGetLastError());
    rc = read_status(c);
    if (rc) return rc;
    const uint32_t fl = c->h_status->flags;
    if (fl & FLAG_BAD_TYPE) return fail(c, DP_E_TYPE, "atom type out of range");
    if (fl & FLAG_KEY_CAP) return fail(c, DP_E_CAP, "more than 512 neighbours within rcut of one atom");
    if (fl & FLAG_CAND_CAP) {
      cap *= 2;
      if (c->timing && c->nev > 0) --c->nev;
      continue;
    }
    c->stats.natoms = n;
    c->stats.evaluations += 1;
    c->stats.cand_cap = c->ws.cand_cap;
    c->cgrid_ok = false;
    return DP_OK;
  }
  c->n_force = 0;
  return fail(c, DP_E_CAP, "candidate list capacity could not be sized");
}

int dp_compute(dp_ctx *c, int64_t n, const double *coords, const int32_t *types, const double *box, double *energy,
               double *forces, double *virial) {
  return compute_impl(c, n, coords, types, box, energy, forces, virial, true);
}

int dp_compute_local(dp_ctx *c, int64_t n_local, int64_t natoms, const double *coords, const int32_t *types,
                     const double *box, double *energy, double *forces, double *virial) {
  const int rc = compute_local_impl(c, n_local, natoms, coords, types, box, energy, forces, virial);
  if (c) c->n_force = 0;
  return rc;
}

int dp_scatter_add_forces(dp_ctx *c, int64_t n, const int32_t *index, const double *f_in, double *f_out) {
  if (!c) return DP_E_ARG;
  if (n < 0 || (n > 0 && (!index || !f_in || !f_out))) return fail(c, DP_E_ARG, "bad scatter arguments");
  HIPCHK(c, hipSetDevice(c->device));
  if (n > 0)
    hipLaunchKernelGGL(k_scatter_add3, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, c->stream, n, index, f_in,
                       f_out);
  HIPCHK(c, hipGetLastError());
  return DP_OK;
}

int dp_compute_noalloc(dp_ctx *c, int64_t n, const double *coords, const int32_t *types, const double *box,
                       double *energy, double *forces, double *virial) {
  if (!c) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "evaluation before dp_set_model");
  if (!c->scratch)
    return fail(c, DP_E_HIP, std::string("dp_compute_noalloc: the static scratch array has no device address: ") +
                                 hipGetErrorString(c->scratch_rc));
  if (c->en[c->active].wide)
    return fail(c, DP_E_MODEL, "dp_compute_noalloc: wide embedding nets (widths above 128) lay out their "
                               "activation buffers per evaluation; use dp_compute");
  // The context's own workspace, and the state that describes its lists and
  // a pending dp_energy, are left as they are.
  const int64_t last_n = c->last_n;
  const bool fwd_ready = c->fwd_ready, cgrid_ok = c->cgrid_ok;
  const CellGrid cgrid = c->cgrid;
  double box_L[3];
  std::memcpy(box_L, c->box_L, sizeof box_L);
  std::swap(c->ws, c->ws_na);
  c->noalloc = true;
  const int rc = compute_impl(c, n, coords, types, box, energy, forces, virial, true);
  c->noalloc = false;
  std::swap(c->ws, c->ws_na);
  c->last_n = last_n;
  c->fwd_ready = fwd_ready;
  c->cgrid_ok = cgrid_ok;
  c->cgrid = cgrid;
  std::memcpy(c->box_L, box_L, sizeof box_L);
  return rc;
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
    tmark(c, 8);
    eval_backward(c, n, F, w.virial);
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
  if (nlist) {
    launch_pad_nlist(c->stream, n, c->dims, c->ws.nreal, c->ws.nlist);
    HIPCHK(c, hipMemcpyAsync(nlist, c->ws.nlist, sizeof(int32_t) * n * c->dims.nnei, hipMemcpyDeviceToDevice,
                             c->stream));
  }
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

int dp_set_wide_storage(dp_ctx *c, int mode) {
  if (!c) return DP_E_ARG;
  if (mode != 0 && mode != 1) return fail(c, DP_E_ARG, "wide storage mode must be 0 (hi + lo) or 1 (16-bit)");
  c->wide_split = mode == 0 ? 1 : 0;
  c->fwd_ready = false;
  return DP_OK;
}

int dp_student_table(dp_ctx *c, int on) {
  if (!c) return DP_E_ARG;
  if ((on != 0) != c->use_tab) c->fwd_ready = false;  // forward and backward would use other layers
  c->use_tab = on != 0;
  return DP_OK;
}

int dp_set_force_scatter(dp_ctx *c, int mode) {
  if (!c) return DP_E_ARG;
  if (mode != 0 && mode != 1) return fail(c, DP_E_ARG, "force scatter mode must be 0 or 1");
  c->scatter = mode;
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
  const bool judging = c->active == 1 && c->judge_every > 0;
  // (Re)start at step st0 from the coordinates and velocities as they are:
  // lists built anew, forces evaluated; at st0 > 0 (a resume after the
  // candidate list was regrown) the step's second half kick follows.
  auto start = [&](int64_t st0) -> int {
    Workspace &w = c->ws;
    F = forces ? forces : w.force_tmp;
    tmark(c, 0);
    hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, w.status, (uint32_t)FLAG_REBUILD);
    launch_wrap(s, n, coords, types, d.ntypes, L, w.xw, &w.status->flags);
    launch_type_sort(s, n, w.xw, d.ntypes, w.blk_counts, w.type_count, w.type_start, w.pos_of_atom, w.atom_of_pos,
                     w.rows_cap);
    build_lists(c, n, g, rlist, &w.status->flags);
    launch_copy_ref(s, n, w.xw, w.xref, &w.status->flags);
    launch_end_rebuild(s, &w.status->flags, &w.status->nbuild);
    eval_body(c, n, L, F);
    if (judging && c->active == 1 && st0 % c->judge_every == 0) {
      const int r = judge_step(c, n, F, st0, L);
      if (r) return r;
    }
    if (st0 > 0)
      launch_verlet_half(s, n, vel, F, types, inv_m, 0.5 * dt, &w.status->flags, &w.status->fault_step, st0);
    if (thermo && st0 % thermo_every == 0) {
      launch_kinetic(s, n, vel, types, mass, w.partial, w.ke);
      launch_thermo_row(s, thermo + 6 * (st0 / thermo_every), (double)st0, w.ke, w.energy, w.virial, ndof_kb, inv3v,
                        &w.status->flags);
    }
    return DP_OK;
  };
  rc = start(0);
  if (rc) return rc;
  int regrown = 0;
  // Read the flags after step st.  A skin-list overflow at a step after the
  // last check stopped the integrator there: the list is grown and the run
  // restarted at that step (*resume); other errors end the run.
  auto check = [&](int64_t st, int64_t &resume) -> int {
    HIPCHK(c, hipGetLastError());
    int r = read_status(c);
    if (r) return r;
    const uint32_t fl = c->h_status->flags;
    if (fl & FLAG_BAD_TYPE) return fail(c, DP_E_TYPE, "atom type out of range");
    if (fl & FLAG_KEY_CAP) return fail(c, DP_E_CAP, "more than 512 neighbours within rcut of one atom");
    if (fl & FLAG_NONFINITE) return fail(c, DP_E_NONFINITE, "non-finite energy by step " + std::to_string(st));
    if (fl & FLAG_CAND_CAP) {
      const long long f0 = nsteps == 0 ? 0 : c->h_status->fault_step;
      if (regrown >= 4 || f0 < 0 || f0 > st)
        return fail(c, DP_E_CAP, "skin candidate list overflow; use a smaller skin");
      ++regrown;
      r = ensure_ws(c, n, ncell, 2 * c->ws.cand_cap);
      if (r) return r;
      r = start((int64_t)f0);
      if (r) return r;
      resume = (int64_t)f0;
    }
    return DP_OK;
  };
  int64_t resume = -1;
  for (int64_t st = 1; st <= nsteps; ++st) {
    Workspace &w = c->ws;
    tmark(c, 0);
    // the first half kick of step st records st - 1 when an error flag
    // stopped the run: the state is then that of the end of step st - 1
    // before its second half kick (or the start, st - 1 = 0)
    launch_verlet_half(s, n, vel, F, types, inv_m, 0.5 * dt, &w.status->flags, &w.status->fault_step, st - 1);
    launch_verlet_drift(s, n, coords, vel, dt, L, &w.status->flags);
    launch_wrap(s, n, coords, types, d.ntypes, L, w.xw, &w.status->flags);
    launch_max_disp(s, n, w.xw, w.xref, L, 0.5 * skin, &w.status->flags);
    build_lists(c, n, g, rlist, &w.status->flags);
    launch_copy_ref(s, n, w.xw, w.xref, &w.status->flags);
    launch_end_rebuild(s, &w.status->flags, &w.status->nbuild);
    eval_body(c, n, L, F);
    if (judging && c->active == 1 && st % c->judge_every == 0) {
      rc = judge_step(c, n, F, st, L);
      if (rc) return rc;
    }
    launch_verlet_half(s, n, vel, F, types, inv_m, 0.5 * dt, &w.status->flags, &w.status->fault_step, st);
    const bool th = thermo && (st % thermo_every == 0);
    if (th) {
      launch_kinetic(s, n, vel, types, mass, w.partial, w.ke);
      launch_thermo_row(s, thermo + 6 * (st / thermo_every), (double)st, w.ke, w.energy, w.virial, ndof_kb, inv3v,
                        &w.status->flags);
    }
    c->stats.evaluations += 1;
    if (th || st == nsteps) {
      resume = -1;
      rc = check(st, resume);
      if (rc) return rc;
      if (resume >= 0) st = resume;
    }
  }
  // a run of no steps, or a restart at the last step, has not been checked
  if (nsteps == 0 || resume == nsteps) {
    for (;;) {
      int64_t again = -1;
      rc = check(nsteps, again);
      if (rc) return rc;
      if (again < 0) break;
    }
  }
  c->stats.natoms = n;
  c->stats.cand_cap = c->ws.cand_cap;
  c->last_n = n;
  return DP_OK;
}

// ---------------------------------------------------------------------------
// student embedding net
// ---------------------------------------------------------------------------
int dp_student_default_cfg(dp_student_cfg *cfg) {
  if (!cfg) return DP_E_ARG;
  cfg->batch = 4096;
  cfg->adam_steps = 500;
  cfg->lr = 1e-3;
  cfg->beta1 = 0.9;
  cfg->beta2 = 0.999;
  cfg->eps = 1e-8;
  cfg->ls_samples = 262144;
  cfg->ridge = 1e-14;
  cfg->seed = 20240607ull;
  cfg->init = 1;
  cfg->refit = 1;
  return DP_OK;
}

int dp_student_train(dp_ctx *c, const dp_student_cfg *cfg, double *fit_rmse) {
  if (!c || !cfg) return DP_E_ARG;
  if (!lists_ready(c)) return fail(c, DP_E_NOMODEL, "dp_student_train needs a preceding evaluation");
  const dp_student_cfg &g = *cfg;
  if (g.batch < 64 || g.batch % 64 != 0 || g.batch > (1 << 20) || g.adam_steps < 0 || !(g.lr > 0) ||
      !(g.beta1 >= 0 && g.beta1 < 1) || !(g.beta2 >= 0 && g.beta2 < 1) || !(g.eps > 0) || !(g.ridge >= 0) ||
      (g.refit && (g.ls_samples < g.batch || g.ls_samples % g.batch != 0)))
    return fail(c, DP_E_ARG, "bad student configuration");
  if (c->dims.M1 > 128) return fail(c, DP_E_MODEL, "student nets need M1 <= 128");
  if (prec16(c->precision) && c->dims.M1 != 100)
    return fail(c, DP_E_MODEL, "the 16-bit student kernels exist for M1 = 100 only");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = ensure_student(c, g.batch);
  if (rc) return rc;
  Student *st = c->st;
  const StudentLayout L = student_layout(st->M1);
  hipStream_t s = c->stream;
  if (g.init || !st->have_params) {
    // scale of the first layer from the largest s of the first batch
    st_draw(c, g.seed, 0, g.batch);
    std::vector<double> sv((size_t)st->nets * g.batch);
    HIPCHK(c, hipMemcpyAsync(sv.data(), st->s, sizeof(double) * sv.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    std::vector<double> smax(st->nets, 0.0);
    for (int net = 0; net < st->nets; ++net)
      for (int64_t q = 0; q < g.batch; ++q) smax[net] = std::max(smax[net], sv[(size_t)net * g.batch + q]);
    std::vector<float> P;
    st_init_params(*st, g.seed, smax, P);
    HIPCHK(c, hipMemcpy(st->params, P.data(), sizeof(float) * P.size(), hipMemcpyHostToDevice));
    launch_fill_u32(s, (uint32_t *)st->m, (int64_t)st->nets * L.np, 0u);
    launch_fill_u32(s, (uint32_t *)st->v, (int64_t)st->nets * L.np, 0u);
    st->have_params = true;
    st->t = 0;
  }
  const int64_t nbmax = st->cap_draw / g.batch;
  for (int64_t k0 = 0; k0 < g.adam_steps; k0 += nbmax) {
    // batches t .. t + nb - 1 (sample indices t * batch ...) in one draw
    const int nb = (int)std::min<int64_t>(nbmax, g.adam_steps - k0);
    st_draw(c, g.seed, st->t * g.batch, g.batch, nb);
    for (int k = 0; k < nb; ++k) {
      st_grad(c, g.batch, k);
      st_adam(c, g.batch, g, nullptr);
      st->t += 1;
    }
  }
  HIPCHK(c, hipGetLastError());
  double result = 0.0;
  if (g.adam_steps > 0) {
    std::vector<double> loss(st->nets);
    HIPCHK(c, hipMemcpyAsync(loss.data(), st->loss, sizeof(double) * st->nets, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (double v : loss) result = std::max(result, v);
  }
  if (g.refit) {
    const int quant = quant_of(c);
    const int NE = SNF * SNF + SNF * st->M1;
    launch_fill_u32(s, (uint32_t *)st->lspart, (int64_t)st->nets * st_ls_blocks() * NE * 2, 0u);
    const int64_t nls = g.ls_samples / g.batch;
    for (int64_t b0 = 0; b0 < nls; b0 += nbmax) {
      const int nb = (int)std::min<int64_t>(nbmax, nls - b0);
      st_draw(c, g.seed, ST_Q_LS + b0 * g.batch, g.batch, nb);
      StLsArgs la{};
      la.M1 = st->M1;
      la.nets = st->nets;
      la.batch = (int)g.batch;
      la.nblk = st_ls_blocks();
      la.nb = nb;
      la.params = st->params;
      la.quant = quant;
      la.s = st->s;
      la.wt = st->wt;
      la.G = st->G;
      la.part = st->lspart;
      launch_st_ls(s, la);
    }
    launch_st_lsfold(s, st->M1, st->nets, st_ls_blocks(), st->lspart, st->lsfold);
    StSolveArgs va{};
    va.M1 = st->M1;
    va.nets = st->nets;
    va.nblk = ST_LS_FOLD;
    va.part = st->lsfold;
    va.ridge = g.ridge;
    va.quant = quant;
    va.X = st->X;
    va.status = st->status;
    launch_st_solve(s, va);
    // held-out check of the fitted model
    st_draw(c, g.seed, ST_Q_CHECK, ST_CHECK_N);
    StCheckArgs ca{};
    ca.M1 = st->M1;
    ca.nets = st->nets;
    ca.batch = (int)ST_CHECK_N;
    ca.params = st->params;
    ca.X = st->X;
    ca.quant = quant;
    ca.s = st->s;
    ca.wt = st->wt;
    ca.G = st->G;
    ca.part = st->chk;
    launch_st_check(s, ca);
    HIPCHK(c, hipGetLastError());
    std::vector<int32_t> stat(st->nets);
    const int64_t ncb = ST_CHECK_N / 64;
    std::vector<double> chk((size_t)st->nets * ncb * 2);
    std::vector<float> P((size_t)st->nets * L.np);
    std::vector<double> X((size_t)st->nets * SNF * st->M1);
    HIPCHK(c, hipMemcpyAsync(stat.data(), st->status, sizeof(int32_t) * stat.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(chk.data(), st->chk, sizeof(double) * chk.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(P.data(), st->params, sizeof(float) * P.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(X.data(), st->X, sizeof(double) * X.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    result = 0.0;
    for (int net = 0; net < st->nets; ++net) {
      if (stat[net] == 2) {
        // no neighbour of this type pair in the frame: the net is never
        // evaluated on it; keep an all-zero output layer
        std::fill(X.begin() + (size_t)net * SNF * st->M1, X.begin() + (size_t)(net + 1) * SNF * st->M1, 0.0);
        continue;
      }
      if (stat[net] != 0)
        return fail(c, DP_E_MODEL, "student least squares: normal matrix not positive definite (net " +
                                       std::to_string(net) + "); raise the ridge");
      double e2 = 0.0, g2 = 0.0;
      for (int64_t b = 0; b < ncb; ++b) {
        e2 += chk[((size_t)net * ncb + b) * 2];
        g2 += chk[((size_t)net * ncb + b) * 2 + 1];
      }
      if (g2 > 0) result = std::max(result, std::sqrt(e2 / g2));
    }
    rc = install_student(c, student_model(c, P, X, quant));
    if (rc) return rc;
  }
  if (fit_rmse) *fit_rmse = result;
  return DP_OK;
}

int dp_student_get_params(dp_ctx *c, float *params) {
  if (!c || !params) return DP_E_ARG;
  if (!c->st || !c->st->have_params) return fail(c, DP_E_NOMODEL, "no student parameters");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(params, c->st->params, sizeof(float) * c->st->nets * c->st->np, hipMemcpyDeviceToHost));
  return DP_OK;
}

int dp_student_set_params(dp_ctx *c, const float *params) {
  if (!c || !params) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "no model");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = ensure_student(c, c->st ? c->st->cap : 4096);
  if (rc) return rc;
  Student *st = c->st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(st->params, params, sizeof(float) * st->nets * st->np, hipMemcpyHostToDevice));
  launch_fill_u32(c->stream, (uint32_t *)st->m, (int64_t)st->nets * st->np, 0u);
  launch_fill_u32(c->stream, (uint32_t *)st->v, (int64_t)st->nets * st->np, 0u);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  st->have_params = true;
  st->t = 0;
  return DP_OK;
}

int dp_student_batch_grad(dp_ctx *c, uint64_t seed, int64_t step, int64_t batch, double *s_out, double *loss,
                          float *grad) {
  if (!c) return DP_E_ARG;
  if (!lists_ready(c)) return fail(c, DP_E_NOMODEL, "dp_student_batch_grad needs a preceding evaluation");
  if (batch < 64 || batch % 64 != 0 || batch > (1 << 20) || step < 0)
    return fail(c, DP_E_ARG, "batch must be a positive multiple of 64");
  if (!c->st || !c->st->have_params) return fail(c, DP_E_NOMODEL, "no student parameters");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = ensure_student(c, batch);
  if (rc) return rc;
  Student *st = c->st;
  hipStream_t s = c->stream;
  dp_student_cfg g;
  dp_student_default_cfg(&g);
  st_draw(c, seed, step * batch, batch);
  st_grad(c, batch);
  st_adam(c, batch, g, st->gout);
  HIPCHK(c, hipGetLastError());
  if (s_out) HIPCHK(c, hipMemcpyAsync(s_out, st->s, sizeof(double) * st->nets * batch, hipMemcpyDeviceToHost, s));
  if (loss) HIPCHK(c, hipMemcpyAsync(loss, st->loss, sizeof(double) * st->nets, hipMemcpyDeviceToHost, s));
  if (grad) HIPCHK(c, hipMemcpyAsync(grad, st->gout, sizeof(float) * st->nets * st->np, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return DP_OK;
}

int dp_student_use(dp_ctx *c, int on) {
  if (!c) return DP_E_ARG;
  if (on && !c->en[1].ready) return fail(c, DP_E_NOMODEL, "no student installed");
  c->active = on ? 1 : 0;
  c->fwd_ready = false;
  return DP_OK;
}

int dp_student_judge(dp_ctx *c, int64_t every, double max_force_rmse) {
  if (!c) return DP_E_ARG;
  if (every < 0 || !(max_force_rmse >= 0)) return fail(c, DP_E_ARG, "bad judge settings");
  c->judge_every = every;
  c->judge_max = max_force_rmse;
  return DP_OK;
}

int dp_student_judge_sample(dp_ctx *c, double side) {
  if (!c) return DP_E_ARG;
  if (!(side >= 0.0) || !std::isfinite(side)) return fail(c, DP_E_ARG, "judge cube side must be >= 0");
  c->judge_side = side;
  return DP_OK;
}

int dp_student_get_model(dp_ctx *c, void *buf, size_t cap, size_t *nbytes) {
  if (!c || !nbytes) return DP_E_ARG;
  if (!c->en[1].ready) return fail(c, DP_E_NOMODEL, "no student installed");
  const std::vector<unsigned char> b = write_blob(c->shm);
  *nbytes = b.size();
  if (buf) std::memcpy(buf, b.data(), std::min(cap, b.size()));
  return DP_OK;
}

int dp_student_set_model(dp_ctx *c, const void *blob, size_t nbytes) {
  if (!c || !blob) return DP_E_ARG;
  if (!c->has_model) return fail(c, DP_E_NOMODEL, "no teacher model");
  HIPCHK(c, hipSetDevice(c->device));
  HostModel m;
  std::string err;
  if (!parse_blob(blob, nbytes, m, err)) return fail(c, DP_E_MODEL, err);
  const HostModel &h = c->hm;
  const bool same = m.ntypes == h.ntypes && m.rcut == h.rcut && m.rcut_smth == h.rcut_smth &&
                    m.desc_norm == h.desc_norm && m.sel == h.sel && m.M2 == h.M2 && m.n_fit == h.n_fit &&
                    m.fit_w == h.fit_w && m.fW == h.fW && m.fb == h.fb;
  if (!same) return fail(c, DP_E_MODEL, "student blob: geometry or fitting nets differ from the teacher's");
  if (!(m.n_emb == 3 && m.emb_lin == 1 && m.emb_w[1] == SH1 && m.emb_w[2] == SH2 && m.emb_w[3] == c->dims.M1))
    return fail(c, DP_E_MODEL, "student blob: embedding must be 1-16-32-M1 with an affine last layer");
  return install_student(c, std::move(m));
}

}  // extern "C"
