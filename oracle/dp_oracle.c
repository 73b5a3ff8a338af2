/*
 * dp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference of the Deep Potential (smooth edition)
 * energy / force / virial evaluation that the paper accelerates
 * (Section III "Deep Potential Molecular Dynamics", Fig. 1; Section V-B,
 * "Increasing computational granularity" and "Optimization of Customized
 * TensorFlow Operators").  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code with the HIP library.
 *
 * Every function follows the plain definition, step by step:
 *   wrap -> neighbour set {j : |r_ij| <= rc}, r_ij = r_j - r_i
 *   -> type-sorted, distance-sorted, sel-padded list (Section V-B: sort by
 *      type, then distance; keep the nearest sel per type; pad with -1;
 *      ties broken by index as in the packed 64-bit key)
 *   -> environment matrix rows (s, s x/r, s y/r, s z/r), s = sw(r)/r
 *   -> embedding net G(s) per (centre type, neighbour type), Fig. 1(c,e,f)
 *   -> T = (1/Nc) sum_j G_j R_j^T,  D = T T_<^T
 *   -> fitting net per centre type, Fig. 1(d,g) -> E_i;  E = sum_i E_i
 *   -> reverse-mode chain rule -> dE/dR_j -> g_ij = dE/dr_ij
 *   -> F_i += g_ij, F_j -= g_ij;  virial Xi = -sum g_ij (x) r_ij.
 * The paper gives these steps in words only; the readings taken where it is
 * silent (switching function, descriptor constant, skip rule, ...) are the
 * ones listed in the design notes of this repository.
 *
 * Built with gcc -O2 -ffp-contract=off (no FMA contraction, no fast-math)
 * so that every distance is the IEEE result of the written operation order.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXT 8
#define OR_MAXL 8
#define OR_WMAX 32768 /* widest layer input or output, D = M1*M2 included */

typedef struct {
  int64_t ntypes, n_emb, n_fit, M2, M1, nnei;
  int64_t emb_lin;                /* 1: the last embedding layer has no tanh */
  double rcut, rcut_smth, desc_norm;
  int64_t sel[OR_MAXT], off[OR_MAXT + 1];
  int64_t emb_w[OR_MAXL + 1];     /* emb_w[0] = 1, emb_w[n_emb] = M1 */
  int64_t fit_w[OR_MAXL + 2];     /* fit_w[0] = M1*M2, ..., fit_w[n_fit+1] = 1 */
  double *eW[OR_MAXT][OR_MAXT][OR_MAXL], *eb[OR_MAXT][OR_MAXT][OR_MAXL];
  double *fW[OR_MAXT][OR_MAXL + 1], *fb[OR_MAXT][OR_MAXL + 1];
  double *store;
} or_model;

static char or_err[256];
const char *or_last_error(void) { return or_err; }

/* threads an evaluation uses (OpenMP default, e.g. OMP_NUM_THREADS) */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* model blob                                                          */
/* ------------------------------------------------------------------ */
static int rd_i64(const unsigned char **p, const unsigned char *end, int64_t *v) {
  if (end - *p < 8) return -1;
  memcpy(v, *p, 8); *p += 8; return 0;
}
static int rd_f64(const unsigned char **p, const unsigned char *end, double *v) {
  if (end - *p < 8) return -1;
  memcpy(v, *p, 8); *p += 8; return 0;
}

void or_model_free(void *h) {
  or_model *m = (or_model *)h;
  if (!m) return;
  free(m->store);
  free(m);
}

void *or_model_new(const void *blob, int64_t nbytes) {
  const unsigned char *p = (const unsigned char *)blob, *end = p + nbytes;
  int64_t ver, t, u, l;
  or_model *m;
  if (nbytes < 8 || memcmp(p, "DPMIBLOB", 8) != 0) { snprintf(or_err, sizeof or_err, "bad magic"); return NULL; }
  p += 8;
  m = (or_model *)calloc(1, sizeof(or_model));
  if (rd_i64(&p, end, &ver) || (ver != 1 && ver != 2)) goto bad;
  if (rd_i64(&p, end, &m->ntypes) || rd_i64(&p, end, &m->n_emb) || rd_i64(&p, end, &m->n_fit) ||
      rd_i64(&p, end, &m->M2)) goto bad;
  /* version 2 adds one flag: a linear (activation-free) last embedding layer */
  if (ver == 2 && (rd_i64(&p, end, &m->emb_lin) || (m->emb_lin != 0 && m->emb_lin != 1))) goto bad;
  if (m->ntypes < 1 || m->ntypes > OR_MAXT || m->n_emb < 1 || m->n_emb > OR_MAXL || m->n_fit < 1 ||
      m->n_fit > OR_MAXL) goto bad;
  if (rd_f64(&p, end, &m->rcut) || rd_f64(&p, end, &m->rcut_smth) || rd_f64(&p, end, &m->desc_norm)) goto bad;
  m->off[0] = 0;
  for (t = 0; t < m->ntypes; ++t) {
    if (rd_i64(&p, end, &m->sel[t]) || m->sel[t] < 0) goto bad;
    m->off[t + 1] = m->off[t] + m->sel[t];
  }
  m->nnei = m->off[m->ntypes];
  for (l = 0; l <= m->n_emb; ++l) if (rd_i64(&p, end, &m->emb_w[l]) || m->emb_w[l] < 1) goto bad;
  if (m->emb_w[0] != 1) goto bad;
  m->M1 = m->emb_w[m->n_emb];
  if (m->M2 < 1 || m->M2 > m->M1) goto bad;
  m->fit_w[0] = m->M1 * m->M2;
  for (l = 1; l <= m->n_fit; ++l) if (rd_i64(&p, end, &m->fit_w[l]) || m->fit_w[l] < 1) goto bad;
  m->fit_w[m->n_fit + 1] = 1;
  for (l = 0; l <= m->n_emb; ++l) if (m->emb_w[l] > OR_WMAX) goto bad;
  for (l = 0; l <= m->n_fit; ++l) if (m->fit_w[l] > OR_WMAX) goto bad;
  {
    int64_t total = 0;
    for (t = 0; t < m->ntypes; ++t)
      for (u = 0; u < m->ntypes; ++u)
        for (l = 0; l < m->n_emb; ++l) total += m->emb_w[l] * m->emb_w[l + 1] + m->emb_w[l + 1];
    for (t = 0; t < m->ntypes; ++t)
      for (l = 0; l <= m->n_fit; ++l) total += m->fit_w[l] * m->fit_w[l + 1] + m->fit_w[l + 1];
    if ((int64_t)(end - p) != total * 8) goto bad;
    m->store = (double *)malloc((size_t)total * sizeof(double));
    memcpy(m->store, p, (size_t)total * 8);
  }
  {
    double *q = m->store;
    for (t = 0; t < m->ntypes; ++t)
      for (u = 0; u < m->ntypes; ++u)
        for (l = 0; l < m->n_emb; ++l) {
          m->eW[t][u][l] = q; q += m->emb_w[l] * m->emb_w[l + 1];
          m->eb[t][u][l] = q; q += m->emb_w[l + 1];
        }
    for (t = 0; t < m->ntypes; ++t)
      for (l = 0; l <= m->n_fit; ++l) {
        m->fW[t][l] = q; q += m->fit_w[l] * m->fit_w[l + 1];
        m->fb[t][l] = q; q += m->fit_w[l + 1];
      }
  }
  return m;
bad:
  snprintf(or_err, sizeof or_err, "malformed model blob");
  free(m);
  return NULL;
}

/* header fields for the Python side: ntypes, n_emb, n_fit, M1, M2, nnei */
void or_model_dims(const void *h, int64_t *out6) {
  const or_model *m = (const or_model *)h;
  out6[0] = m->ntypes; out6[1] = m->n_emb; out6[2] = m->n_fit;
  out6[3] = m->M1; out6[4] = m->M2; out6[5] = m->nnei;
}

/* ------------------------------------------------------------------ */
/* geometry: wrapping, minimum image, distance                          */
/* ------------------------------------------------------------------ */
/* x <- x - L floor(x/L); a result equal to L (from rounding) becomes 0. */
static double or_wrap1(double x, double L) {
  double y = x - L * floor(x / L);
  if (y >= L) y = 0.0;
  return y;
}

void or_wrap(int64_t n, const double *x, const double *box, double *xw) {
  int64_t i;
  int a;
  for (i = 0; i < n; ++i)
    for (a = 0; a < 3; ++a) xw[3 * i + a] = or_wrap1(x[3 * i + a], box[a]);
}

/* Minimum-image displacement d = r_j - r_i (orthorhombic, one correction)
 * and r = sqrt((dx dx + dy dy) + dz dz), evaluated in exactly this order. */
static double or_disp(const double *xi, const double *xj, const double *L, double *d) {
  int a;
  double r2;
  for (a = 0; a < 3; ++a) {
    double v = xj[a] - xi[a];
    if (v > 0.5 * L[a]) v -= L[a];
    else if (v < -0.5 * L[a]) v += L[a];
    d[a] = v;
  }
  r2 = d[0] * d[0] + d[1] * d[1];
  r2 = r2 + d[2] * d[2];
  return sqrt(r2);
}

/* ------------------------------------------------------------------ */
/* neighbour list: Section V-B formatting                              */
/* ------------------------------------------------------------------ */
typedef struct { int64_t type; uint64_t q; int64_t j; } or_key;

static int or_key_cmp(const void *a, const void *b) {
  const or_key *x = (const or_key *)a, *y = (const or_key *)b;
  if (x->type != y->type) return x->type < y->type ? -1 : 1;
  if (x->q != y->q) return x->q < y->q ? -1 : 1;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  return 0;
}

/* Format one centre's candidate set: keep r <= rc, sort by the key
 * (type, floor(r * 1e8), j), keep the first sel_u of each type, pad -1. */
static void or_format_row(const or_model *m, int64_t i, const double *xw, const int32_t *types,
                          const double *box, const int64_t *cand, int64_t ncand, or_key *buf,
                          int32_t *row, int32_t *nreal, int64_t *overflow) {
  int64_t c, k = 0, u;
  for (c = 0; c < ncand; ++c) {
    int64_t j = cand[c];
    double d[3], r;
    if (j == i) continue;
    r = or_disp(&xw[3 * i], &xw[3 * j], box, d);
    if (r <= m->rcut) {
      buf[k].type = types[j];
      buf[k].q = (uint64_t)floor(r * 1e8);
      buf[k].j = j;
      ++k;
    }
  }
  qsort(buf, (size_t)k, sizeof(or_key), or_key_cmp);
  for (c = 0; c < m->nnei; ++c) row[c] = -1;
  {
    int64_t cnt[OR_MAXT] = {0};
    for (c = 0; c < k; ++c) {
      u = buf[c].type;
      if (cnt[u] < m->sel[u]) row[m->off[u] + cnt[u]] = (int32_t)buf[c].j;
      cnt[u]++;
    }
    for (u = 0; u < m->ntypes; ++u) {
      nreal[u] = (int32_t)(cnt[u] < m->sel[u] ? cnt[u] : m->sel[u]);
      if (cnt[u] > m->sel[u]) *overflow += cnt[u] - m->sel[u];
    }
  }
}

/* Cell grid with side >= rc: nc = floor(L / (rc + 1e-6)), at least 1. */
typedef struct { int nc[3]; int64_t *start, *idx; } or_cells;

static void or_cells_build(or_cells *cl, int64_t n, const double *xw, const double *box, double rc) {
  int a;
  int64_t i, ncell, *cnt;
  for (a = 0; a < 3; ++a) {
    cl->nc[a] = (int)floor(box[a] / (rc + 1e-6));
    if (cl->nc[a] < 1) cl->nc[a] = 1;
  }
  ncell = (int64_t)cl->nc[0] * cl->nc[1] * cl->nc[2];
  cl->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  cl->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  cnt = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
  for (i = 0; i < n; ++i) {
    int64_t c[3];
    for (a = 0; a < 3; ++a) {
      c[a] = (int64_t)floor(xw[3 * i + a] / (box[a] / cl->nc[a]));
      if (c[a] >= cl->nc[a]) c[a] = cl->nc[a] - 1;
      if (c[a] < 0) c[a] = 0;
    }
    cl->start[(c[0] * cl->nc[1] + c[1]) * cl->nc[2] + c[2] + 1]++;
  }
  for (i = 0; i < ncell; ++i) cl->start[i + 1] += cl->start[i];
  for (i = 0; i < n; ++i) {
    int64_t c[3], id;
    for (a = 0; a < 3; ++a) {
      c[a] = (int64_t)floor(xw[3 * i + a] / (box[a] / cl->nc[a]));
      if (c[a] >= cl->nc[a]) c[a] = cl->nc[a] - 1;
      if (c[a] < 0) c[a] = 0;
    }
    id = (c[0] * cl->nc[1] + c[1]) * cl->nc[2] + c[2];
    cl->idx[cl->start[id] + cnt[id]++] = i;
  }
  free(cnt);
}

/* Candidates of atom i from its own and adjacent cells (each distinct
 * periodic cell once, also when a dimension has fewer than 3 cells). */
static int64_t or_cells_cand(const or_cells *cl, const double *xi, const double *box, int64_t *out) {
  int a, o[3][3], no[3];
  int64_t c0[3], k = 0;
  for (a = 0; a < 3; ++a) {
    int t, cnt = 0;
    c0[a] = (int64_t)floor(xi[a] / (box[a] / cl->nc[a]));
    if (c0[a] >= cl->nc[a]) c0[a] = cl->nc[a] - 1;
    if (c0[a] < 0) c0[a] = 0;
    for (t = -1; t <= 1; ++t) {
      int v = (int)(((c0[a] + t) % cl->nc[a] + cl->nc[a]) % cl->nc[a]), dup = 0, s;
      for (s = 0; s < cnt; ++s) if (o[a][s] == v) dup = 1;
      if (!dup) o[a][cnt++] = v;
    }
    no[a] = cnt;
  }
  {
    int x, y, z;
    for (x = 0; x < no[0]; ++x)
      for (y = 0; y < no[1]; ++y)
        for (z = 0; z < no[2]; ++z) {
          int64_t id = ((int64_t)o[0][x] * cl->nc[1] + o[1][y]) * cl->nc[2] + o[2][z], p;
          for (p = cl->start[id]; p < cl->start[id + 1]; ++p) out[k++] = cl->idx[p];
        }
  }
  return k;
}

static int or_check_box(const or_model *m, const double *box) {
  int a;
  for (a = 0; a < 3; ++a)
    if (!(box[a] > 2.0 * m->rcut)) {
      snprintf(or_err, sizeof or_err, "box length %g must exceed 2*rcut", box[a]);
      return -4;
    }
  return 0;
}

/* Formatted list for the given centres (NULL = all atoms, in order).
 * nlist [ncentres][nnei], nreal [ncentres][ntypes].  use_cells selects the
 * cell-list candidate search; 0 is O(N^2) brute force.  Both must agree. */
int or_nlist(const void *h, int64_t n, const double *x, const int32_t *types, const double *box,
             const int64_t *centres, int64_t ncentres, int use_cells, int32_t *nlist, int32_t *nreal,
             int64_t *overflow) {
  const or_model *m = (const or_model *)h;
  double *xw;
  or_cells cl;
  int64_t c, ovf = 0;
  int rc = or_check_box(m, box);
  if (rc) return rc;
  for (c = 0; c < n; ++c)
    if (types[c] < 0 || types[c] >= m->ntypes) { snprintf(or_err, sizeof or_err, "type out of range"); return -5; }
  if (!centres) ncentres = n;
  xw = (double *)malloc((size_t)(n > 0 ? 3 * n : 1) * sizeof(double));
  or_wrap(n, x, box, xw);
  if (use_cells) or_cells_build(&cl, n, xw, box, m->rcut);
#pragma omp parallel reduction(+ : ovf)
  {
    int64_t *cand = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    or_key *buf = (or_key *)malloc((size_t)(n > 0 ? n : 1) * sizeof(or_key));
    int64_t cc;
#pragma omp for schedule(static)
    for (cc = 0; cc < ncentres; ++cc) {
      int64_t i = centres ? centres[cc] : cc, nc, j;
      if (use_cells) nc = or_cells_cand(&cl, &xw[3 * i], box, cand);
      else { for (j = 0; j < n; ++j) cand[j] = j; nc = n; }
      or_format_row(m, i, xw, types, box, cand, nc, buf, &nlist[cc * m->nnei], &nreal[cc * m->ntypes], &ovf);
    }
    free(cand);
    free(buf);
  }
  if (use_cells) { free(cl.start); free(cl.idx); }
  free(xw);
  *overflow = ovf;
  return 0;
}

/* ------------------------------------------------------------------ */
/* environment matrix row and its Jacobian                              */
/* ------------------------------------------------------------------ */
/* Quintic switch, C2 at both ends: sw = 1 below rcs,
 * u^3 (-6u^2 + 15u - 10) + 1 on [rcs, rc), 0 from rc on; u = (r-rcs)/(rc-rcs). */
static void or_switch(double r, double rcs, double rc, double *sw, double *dsw) {
  if (r < rcs) { *sw = 1.0; *dsw = 0.0; return; }
  if (r >= rc) { *sw = 0.0; *dsw = 0.0; return; }
  {
    double u = (r - rcs) / (rc - rcs);
    *sw = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0;
    *dsw = (u * u * (-30.0 * u * u + 60.0 * u - 30.0)) / (rc - rcs);
  }
}

/* R = (s, s dx/r, s dy/r, s dz/r), s = sw/r; J[k][b] = dR[k]/dd[b]. */
static void or_env_row(const double *d, double r, double rcs, double rc, double *R, double *J) {
  double sw, dsw, s, ds, t, dt;
  int a, b;
  or_switch(r, rcs, rc, &sw, &dsw);
  s = sw / r;
  ds = (dsw * r - sw) / (r * r);          /* d s / d r        */
  t = sw / (r * r);                       /* s / r            */
  dt = dsw / (r * r) - 2.0 * sw / (r * r * r);
  R[0] = s;
  for (a = 0; a < 3; ++a) R[1 + a] = t * d[a];
  if (J) {
    for (b = 0; b < 3; ++b) J[b] = ds * d[b] / r;
    for (a = 0; a < 3; ++a)
      for (b = 0; b < 3; ++b) J[(1 + a) * 3 + b] = dt * d[b] / r * d[a] + (a == b ? t : 0.0);
  }
}

/* exported for the pins: one row and its Jacobian for displacement d */
void or_env_single(const void *h, const double *d, double *R, double *J) {
  const or_model *m = (const or_model *)h;
  double r2 = d[0] * d[0] + d[1] * d[1];
  r2 = r2 + d[2] * d[2];
  or_env_row(d, sqrt(r2), m->rcut_smth, m->rcut, R, J);
}

/* ------------------------------------------------------------------ */
/* networks: Fig. 1(e) dense, (f) doubling skip, (g) identity skip        */
/* ------------------------------------------------------------------ */
/* One hidden layer: z = h W + b, t = tanh(z) (t = z for a linear layer);
 * out == in: h' = h + t;  out == 2 in: h' = (h, h) + t;  else h' = t. */
static void or_layer_fwd(const double *W, const double *b, int64_t in, int64_t out, const double *h,
                         double *t, double *hn, int lin) {
  int64_t i, o;
  for (o = 0; o < out; ++o) {
    double z = b[o];
    for (i = 0; i < in; ++i) z += h[i] * W[i * out + o];
    t[o] = lin ? z : tanh(z);
  }
  for (o = 0; o < out; ++o) {
    if (out == in) hn[o] = h[o] + t[o];
    else if (out == 2 * in) hn[o] = h[o % in] + t[o];
    else hn[o] = t[o];
  }
}

/* given dE/dh' and t, return dE/dh */
static void or_layer_bwd(const double *W, int64_t in, int64_t out, const double *t, const double *gh_out,
                         double *gz, double *gh_in, int lin) {
  int64_t i, o;
  for (o = 0; o < out; ++o) gz[o] = lin ? gh_out[o] : gh_out[o] * (1.0 - t[o] * t[o]);
  for (i = 0; i < in; ++i) {
    double g = 0.0;
    for (o = 0; o < out; ++o) g += W[i * out + o] * gz[o];
    if (out == in) g += gh_out[i];
    else if (out == 2 * in) g += gh_out[i] + gh_out[i + in];
    gh_in[i] = g;
  }
}


/* Embedding net of pair (t,u) at input s; stores per-layer tanh outputs in
 * tt (row l at tt + l*OR_WMAX) and per-layer inputs in hh.  G -> out. */
static void or_embed_fwd(const or_model *m, int t, int u, double s, double *hh, double *tt, double *G) {
  int64_t l;
  hh[0] = s;
  for (l = 0; l < m->n_emb; ++l)
    or_layer_fwd(m->eW[t][u][l], m->eb[t][u][l], m->emb_w[l], m->emb_w[l + 1], hh + l * OR_WMAX,
                 tt + l * OR_WMAX, hh + (l + 1) * OR_WMAX, m->emb_lin && l == m->n_emb - 1);
  memcpy(G, hh + m->n_emb * OR_WMAX, (size_t)m->M1 * sizeof(double));
}

/* dE/ds from dE/dG using the stored activations. */
static double or_embed_bwd(const or_model *m, int t, int u, const double *tt, const double *gG, double *w1,
                           double *w2, double *gz) {
  int64_t l;
  memcpy(w1, gG, (size_t)m->M1 * sizeof(double));
  for (l = m->n_emb - 1; l >= 0; --l) {
    or_layer_bwd(m->eW[t][u][l], m->emb_w[l], m->emb_w[l + 1], tt + l * OR_WMAX, w1, gz, w2,
                 m->emb_lin && l == m->n_emb - 1);
    memcpy(w1, w2, (size_t)m->emb_w[l] * sizeof(double));
  }
  return w1[0];
}

/* exported for the pins: G(s) and dG/ds (central difference is the caller's) */
void or_embed_single(const void *h, int t, int u, double s, double *G) {
  const or_model *m = (const or_model *)h;
  double *hh = (double *)malloc((OR_MAXL + 1) * OR_WMAX * sizeof(double));
  double *tt = (double *)malloc((OR_MAXL + 1) * OR_WMAX * sizeof(double));
  or_embed_fwd(m, t, u, s, hh, tt, G);
  free(hh);
  free(tt);
}

/* Fitting net of type t: hidden layers by the same skip rule, then the
 * linear 1-wide output layer.  Returns E_i; keeps activations. */
static double or_fit_fwd(const or_model *m, int t, const double *Dv, double *hh, double *tt) {
  int64_t l, i;
  int64_t L = m->n_fit;
  double e;
  memcpy(hh, Dv, (size_t)m->fit_w[0] * sizeof(double));
  for (l = 0; l < L; ++l)
    or_layer_fwd(m->fW[t][l], m->fb[t][l], m->fit_w[l], m->fit_w[l + 1], hh + l * OR_WMAX,
                 tt + l * OR_WMAX, hh + (l + 1) * OR_WMAX, 0);
  e = m->fb[t][L][0];
  for (i = 0; i < m->fit_w[L]; ++i) e += hh[L * OR_WMAX + i] * m->fW[t][L][i];
  return e;
}

static void or_fit_bwd(const or_model *m, int t, const double *tt, double *gD, double *w1, double *w2,
                       double *gz) {
  int64_t l, i, L = m->n_fit;
  for (i = 0; i < m->fit_w[L]; ++i) w1[i] = m->fW[t][L][i];
  for (l = L - 1; l >= 0; --l) {
    or_layer_bwd(m->fW[t][l], m->fit_w[l], m->fit_w[l + 1], tt + l * OR_WMAX, w1, gz, w2, 0);
    memcpy(w1, w2, (size_t)m->fit_w[l] * sizeof(double));
  }
  memcpy(gD, w1, (size_t)m->fit_w[0] * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* full evaluation                                                      */
/* ------------------------------------------------------------------ */
/* Energy, forces and virial of the atoms in `centres` (NULL = all atoms):
 *   energy = sum over centres of E_i;  force = -d(energy)/dx  [n][3];
 *   virial[9] = -sum_{centres i, j} g_ij (x) r_ij (row-major alpha, beta).
 * Optional per-centre outputs (NULL to skip), rows in centre order:
 *   atom_e [nc], nlist [nc][nnei], nreal [nc][ntypes], rt [nc][nnei][4],
 *   T [nc][M1][4], D [nc][M1*M2], dD [nc][M1*M2], net_deriv [nc][nnei][4]
 *   (net_deriv = dE_i/dR_j including the embedding-net path; padded 0).
 * nthreads <= 0 keeps the OpenMP default.  Force and virial partial sums
 * are per thread and added in thread order.  Returns 0 or a negative code. */
int or_eval(const void *h, int64_t n, const double *x, const int32_t *types, const double *box,
            const int64_t *centres, int64_t ncentres, int nthreads, double *energy, double *force,
            double *virial, double *atom_e, int32_t *nlist_out, int32_t *nreal_out, double *rt_out,
            double *T_out, double *D_out, double *dD_out, double *nd_out, int64_t *overflow_out) {
  const or_model *m = (const or_model *)h;
  int64_t nc, nnei = m->nnei, M1 = m->M1, M2 = m->M2, DD = m->M1 * m->M2;
  int32_t *nlist, *nreal;
  double *xw, *ae, *fbuf, *vbuf;
  int nth = 1, rc, th;
  int64_t ovf = 0, i, k;
  double inv_nc = 1.0 / m->desc_norm;

  rc = or_check_box(m, box);
  if (rc) return rc;
  if (!centres) ncentres = n;
  nc = ncentres;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  nth = omp_get_max_threads();
#endif
  nlist = (int32_t *)malloc((size_t)(nc > 0 ? nc * nnei : 1) * sizeof(int32_t));
  nreal = (int32_t *)malloc((size_t)(nc > 0 ? nc * m->ntypes : 1) * sizeof(int32_t));
  rc = or_nlist(h, n, x, types, box, centres, ncentres, 1, nlist, nreal, &ovf);
  if (rc) { free(nlist); free(nreal); return rc; }
  xw = (double *)malloc((size_t)(n > 0 ? 3 * n : 1) * sizeof(double));
  or_wrap(n, x, box, xw);
  ae = (double *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
  fbuf = (double *)calloc((size_t)nth * (size_t)(3 * n > 0 ? 3 * n : 1), sizeof(double));
  vbuf = (double *)calloc((size_t)nth * 9, sizeof(double));

#pragma omp parallel
  {
    int tid = 0;
    double *hh = (double *)malloc((OR_MAXL + 2) * OR_WMAX * sizeof(double));
    double *tt = (double *)malloc((OR_MAXL + 2) * OR_WMAX * sizeof(double));
    double *fh = (double *)malloc((OR_MAXL + 2) * OR_WMAX * sizeof(double));
    double *ft = (double *)malloc((OR_MAXL + 2) * OR_WMAX * sizeof(double));
    double *w1 = (double *)malloc(OR_WMAX * sizeof(double));
    double *w2 = (double *)malloc(OR_WMAX * sizeof(double));
    double *gz = (double *)malloc(OR_WMAX * sizeof(double));
    double *G = (double *)malloc(OR_WMAX * sizeof(double));
    double *gG = (double *)malloc(OR_WMAX * sizeof(double));
    double *T = (double *)malloc((size_t)M1 * 4 * sizeof(double));
    double *dT = (double *)malloc((size_t)M1 * 4 * sizeof(double));
    double *Dv = (double *)malloc((size_t)DD * sizeof(double));
    double *gD = (double *)malloc((size_t)DD * sizeof(double));
    double *fl, *vl;
    int64_t cc;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    fl = fbuf + (size_t)tid * 3 * n;
    vl = vbuf + (size_t)tid * 9;
#pragma omp for schedule(static)
    for (cc = 0; cc < nc; ++cc) {
      int64_t ii = centres ? centres[cc] : cc;
      int ti = types[ii];
      int64_t u, p, a, b, kk;
      const int32_t *row = &nlist[cc * nnei];
      const int32_t *nr = &nreal[cc * m->ntypes];
      double Ei;
      /* T = (1/Nc) sum over real neighbours of G_j R_j^T */
      memset(T, 0, (size_t)M1 * 4 * sizeof(double));
      for (u = 0; u < m->ntypes; ++u)
        for (p = 0; p < nr[u]; ++p) {
          int64_t slot = m->off[u] + p, j = row[slot];
          double d[3], r, R[4];
          r = or_disp(&xw[3 * ii], &xw[3 * j], box, d);
          or_env_row(d, r, m->rcut_smth, m->rcut, R, NULL);
          or_embed_fwd(m, ti, (int)u, R[0], hh, tt, G);
          for (a = 0; a < M1; ++a)
            for (kk = 0; kk < 4; ++kk) T[a * 4 + kk] += G[a] * R[kk];
          if (rt_out)
            for (kk = 0; kk < 4; ++kk) rt_out[(cc * nnei + slot) * 4 + kk] = R[kk];
        }
      for (a = 0; a < M1 * 4; ++a) T[a] *= inv_nc;
      /* D[a][b] = sum_k T[a][k] T[b][k], b < M2 */
      for (a = 0; a < M1; ++a)
        for (b = 0; b < M2; ++b) {
          double s = 0.0;
          for (kk = 0; kk < 4; ++kk) s += T[a * 4 + kk] * T[b * 4 + kk];
          Dv[a * M2 + b] = s;
        }
      Ei = or_fit_fwd(m, ti, Dv, fh, ft);
      ae[cc] = Ei;
      or_fit_bwd(m, ti, ft, gD, w1, w2, gz);
      /* dT = dD T_<  ;  dT[0:M2] += dD^T T */
      for (a = 0; a < M1; ++a)
        for (kk = 0; kk < 4; ++kk) {
          double s = 0.0;
          for (b = 0; b < M2; ++b) s += gD[a * M2 + b] * T[b * 4 + kk];
          dT[a * 4 + kk] = s;
        }
      for (b = 0; b < M2; ++b)
        for (kk = 0; kk < 4; ++kk) {
          double s = 0.0;
          for (a = 0; a < M1; ++a) s += gD[a * M2 + b] * T[a * 4 + kk];
          dT[b * 4 + kk] += s;
        }
      if (T_out) memcpy(&T_out[cc * M1 * 4], T, (size_t)M1 * 4 * sizeof(double));
      if (D_out) memcpy(&D_out[cc * DD], Dv, (size_t)DD * sizeof(double));
      if (dD_out) memcpy(&dD_out[cc * DD], gD, (size_t)DD * sizeof(double));
      /* per neighbour: dE/dR_j, then g_ij through the Jacobian */
      for (u = 0; u < m->ntypes; ++u)
        for (p = 0; p < nr[u]; ++p) {
          int64_t slot = m->off[u] + p, j = row[slot];
          double d[3], r, R[4], J[12], gR[4], g[3];
          r = or_disp(&xw[3 * ii], &xw[3 * j], box, d);
          or_env_row(d, r, m->rcut_smth, m->rcut, R, J);
          or_embed_fwd(m, ti, (int)u, R[0], hh, tt, G);
          for (kk = 0; kk < 4; ++kk) {
            double s = 0.0;
            for (a = 0; a < M1; ++a) s += G[a] * dT[a * 4 + kk];
            gR[kk] = s * inv_nc;
          }
          for (a = 0; a < M1; ++a) {
            double s = 0.0;
            for (kk = 0; kk < 4; ++kk) s += dT[a * 4 + kk] * R[kk];
            gG[a] = s * inv_nc;
          }
          gR[0] += or_embed_bwd(m, ti, (int)u, tt, gG, w1, w2, gz);
          if (nd_out)
            for (kk = 0; kk < 4; ++kk) nd_out[(cc * nnei + slot) * 4 + kk] = gR[kk];
          for (b = 0; b < 3; ++b) {
            double s = 0.0;
            for (kk = 0; kk < 4; ++kk) s += gR[kk] * J[kk * 3 + b];
            g[b] = s;
          }
          for (b = 0; b < 3; ++b) {
            fl[3 * ii + b] += g[b];
            fl[3 * j + b] -= g[b];
          }
          for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) vl[a * 3 + b] -= g[a] * d[b];
        }
    }
    free(hh); free(tt); free(fh); free(ft); free(w1); free(w2); free(gz);
    free(G); free(gG); free(T); free(dT); free(Dv); free(gD);
  }
  {
    double e = 0.0;
    for (i = 0; i < nc; ++i) e += ae[i];
    *energy = e;
  }
  for (i = 0; i < 3 * n; ++i) {
    double s = 0.0;
    for (th = 0; th < nth; ++th) s += fbuf[(size_t)th * 3 * n + i];
    force[i] = s;
  }
  for (k = 0; k < 9; ++k) {
    double s = 0.0;
    for (th = 0; th < nth; ++th) s += vbuf[th * 9 + k];
    virial[k] = s;
  }
  if (atom_e) memcpy(atom_e, ae, (size_t)nc * sizeof(double));
  if (nlist_out) memcpy(nlist_out, nlist, (size_t)nc * nnei * sizeof(int32_t));
  if (nreal_out) memcpy(nreal_out, nreal, (size_t)nc * m->ntypes * sizeof(int32_t));
  if (overflow_out) *overflow_out = ovf;
  free(nlist); free(nreal); free(xw); free(ae); free(fbuf); free(vbuf);
  return 0;
}

/* ------------------------------------------------------------------ */
/* velocity Verlet (units A, fs, amu, eV)                               */
/* ------------------------------------------------------------------ */
#define OR_MVV2E 103.642696562
#define OR_KB 8.617333262e-5

/* nsteps of: v += dt/2 F/m; x += dt v; wrap; F = F(x); v += dt/2 F/m.
 * thermo [nsteps/every + 1][6] = (step, KE, PE, KE+PE, T, P), P in eV/A^3,
 * P = (2 KE + tr Xi) / (3 V); row 0 is the start.  x, v are updated. */
int or_verlet(const void *h, int64_t n, double *x, double *v, const int32_t *types, const double *box,
              const double *mass_t, double dt, int64_t nsteps, int64_t every, int nthreads, double *thermo) {
  double *f = (double *)malloc((size_t)(3 * n > 0 ? 3 * n : 1) * sizeof(double));
  double e, vir[9], vol = box[0] * box[1] * box[2];
  int64_t s, i, row = 0;
  int a, rc;
  rc = or_eval(h, n, x, types, box, NULL, 0, nthreads, &e, f, vir, NULL, NULL, NULL, NULL, NULL, NULL,
               NULL, NULL, NULL);
  if (rc) { free(f); return rc; }
  for (s = 0; s <= nsteps; ++s) {
    if (s > 0) {
      for (i = 0; i < n; ++i)
        for (a = 0; a < 3; ++a) {
          v[3 * i + a] += 0.5 * dt * f[3 * i + a] / (mass_t[types[i]] * OR_MVV2E);
          x[3 * i + a] = or_wrap1(x[3 * i + a] + dt * v[3 * i + a], box[a]);
        }
      rc = or_eval(h, n, x, types, box, NULL, 0, nthreads, &e, f, vir, NULL, NULL, NULL, NULL, NULL, NULL,
                   NULL, NULL, NULL);
      if (rc) { free(f); return rc; }
      for (i = 0; i < n; ++i)
        for (a = 0; a < 3; ++a) v[3 * i + a] += 0.5 * dt * f[3 * i + a] / (mass_t[types[i]] * OR_MVV2E);
    }
    if (thermo && every > 0 && s % every == 0) {
      double ke = 0.0;
      for (i = 0; i < n; ++i)
        for (a = 0; a < 3; ++a) ke += 0.5 * mass_t[types[i]] * v[3 * i + a] * v[3 * i + a];
      ke *= OR_MVV2E;
      thermo[row * 6 + 0] = (double)s;
      thermo[row * 6 + 1] = ke;
      thermo[row * 6 + 2] = e;
      thermo[row * 6 + 3] = ke + e;
      thermo[row * 6 + 4] = 2.0 * ke / ((3.0 * n - 3.0) * OR_KB);
      thermo[row * 6 + 5] = (2.0 * ke + vir[0] + vir[4] + vir[8]) / (3.0 * vol);
      ++row;
    }
  }
  free(f);
  return 0;
}
