/*
 * dpmi.h -- C ABI of the MI355X (gfx950) Deep Potential evaluator.
 *
 * The library computes, for a periodic orthorhombic box of atoms, the Deep
 * Potential energy E = sum_i E_i, the forces F = -dE/dr and the virial
 * Xi = -sum_{i,j} g_ij (x) r_ij, the quantities the paper's MD step spends
 * its time on (Section III, "Deep Potential Molecular Dynamics" and Fig. 1;
 * Section V-A on the neighbour-list format and the custom Environment,
 * ProdForce and ProdVirial operators; Section V-A "Mixed-precision
 * computation" for the precision modes).  Every step runs in hand-written
 * HIP kernels on the stream given to dp_create.
 *
 * Conventions
 *   - All functions return 0 (DP_OK) or a negative DP_E_* code; no C++
 *     exception crosses this boundary.  dp_last_error() describes the last
 *     failure of a context.
 *   - Units: A, eV, fs, amu.  Arrays are row-major, C order.
 *   - Pointers documented as "device" must be device memory of the
 *     context's GPU (e.g. torch CUDA tensor data_ptr()).  The caller owns
 *     every array it passes; the library owns the model weights it copies
 *     and a workspace that grows to the largest system seen and is then
 *     reused, so steady-state calls allocate nothing.
 *   - Work is enqueued on the context's stream.  dp_compute synchronises
 *     that stream once, at its end, to read its error flags (bad type,
 *     capacity overflow); outputs are valid when it returns DP_OK.
 *   - A context is not thread safe; use one per host thread and stream.
 */
#ifndef DPMI_H
#define DPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_ctx dp_ctx;

enum {
  DP_OK = 0,
  DP_E_ARG = -1,       /* NULL pointer, negative size, bad enum value       */
  DP_E_NOMODEL = -2,   /* dp_compute before dp_set_model                    */
  DP_E_MODEL = -3,     /* malformed blob or shape the kernels do not cover  */
  DP_E_BOX = -4,       /* non-orthorhombic box, or a length <= 2 (rc+skin)  */
  DP_E_TYPE = -5,      /* an atom type outside [0, ntypes)                  */
  DP_E_OOM = -6,       /* device allocation failed                          */
  DP_E_HIP = -7,       /* a HIP runtime call failed                         */
  DP_E_NONFINITE = -8, /* non-finite energy (MD driver)                     */
  DP_E_CAP = -9        /* more neighbours within rc of one atom than the
                          per-atom sort buffer (1024) holds                 */
};

/* Precision policies (after the paper's MIX-16 scheme, Section V-A
 * "Mixed-precision computation").
 * DP_FP64: everything in double.
 * DP_MIX_FP16 / DP_MIX_BF16: embedding layers after the first and the first
 *   two fitting layers as 16-bit matrix-core products with FP32
 *   accumulation and 16-bit weights; activations enter those products as
 *   hi + lo 16-bit pairs (about 22 bits); tanh, the descriptor contractions,
 *   the remaining fitting layers and the output layer in FP32.
 * Coordinates, wrapping, distances, the environment matrix, the force
 * Jacobian, energy / force / virial sums and the integrator stay double in
 * every mode.  (Value 1 is reserved.) */
enum { DP_FP64 = 0, DP_MIX_FP16 = 2, DP_MIX_BF16 = 3 };

typedef struct {
  int64_t natoms;            /* atoms in the last dp_compute                 */
  int64_t sel_overflow;      /* neighbours dropped by the nearest-sel rule   */
  int32_t max_real[8];       /* largest real-neighbour count per type        */
  int64_t nlist_builds;      /* candidate-list (skin) rebuilds so far         */
  int64_t evaluations;       /* energy/force evaluations so far              */
  int64_t cand_cap;          /* candidate slots per atom in the skin list    */
  int64_t student_evals;     /* evaluations that used the student net        */
  int64_t teacher_fallbacks; /* judge rejections of the student net          */
  double last_judge_rmse;    /* force RMSE student vs teacher, eV/A          */
} dp_stats;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the null stream).  *out receives the context. */
int dp_create(dp_ctx **out, int device, void *hip_stream);

/* Load a model blob (host memory, `nbytes` bytes, layout DPMIBLOB v1: magic,
 * int64 version/ntypes/n_emb/n_fit/M2, float64 rcut/rcut_smth/desc_norm,
 * int64 sel[ntypes], emb widths, fit widths, then float64 weights) and keep
 * it on the device in `precision` (DP_FP64 ...).  The blob may be freed
 * after the call.  The descriptor is D = T T_<^T with
 * T = (1/desc_norm) sum_j G(s_j) R_j^T (Fig. 1(b)); one embedding net per
 * (centre type, neighbour type) pair and one fitting net per centre type. */
int dp_set_model(dp_ctx *c, const void *blob, size_t nbytes, int precision);

/* Change the precision policy of the loaded model (weights are re-cast
 * from the double copy). */
int dp_set_precision(dp_ctx *c, int precision);

/* One evaluation.
 *   coords [natoms][3] device, double, A (any periodic image)
 *   types  [natoms]    device, int32, 0..ntypes-1
 *   box    [9]         host, double, row-major cell vectors; must be
 *                      diagonal (orthorhombic) with each length > 2 rc
 *   energy [1]         device, double, eV           (may be NULL)
 *   forces [natoms][3] device, double, eV/A         (may be NULL)
 *   virial [9]         device, double, eV, row-major Xi_ab (may be NULL)
 * The neighbour list is built from scratch (cell list, cutoff rc, no skin),
 * formatted as in Section V-A (type-sorted, then by distance with ties by
 * index, nearest sel kept per type, -1 padded). */
int dp_compute(dp_ctx *c, int64_t natoms, const double *coords, const int32_t *types, const double *box,
               double *energy, double *forces, double *virial);

/* The two halves of dp_compute, for reverse-mode frameworks
 * (torch.autograd.Function): dp_energy runs the forward half only (list,
 * environment matrix, embedding + descriptor, fitting net, energy) and keeps
 * its intermediates; dp_energy_backward then runs the adjoint (fitting-net
 * backward, embedding backward with the force and virial scatter, the
 * paper's ProdForce / ProdVirial) for the same configuration and writes
 *   forces = -grad_energy * dE/dr   (device [natoms][3], may be NULL)
 *   virial = grad_energy * Xi       (device [9], may be NULL).
 * dp_energy_backward may be called again with another grad_energy; any
 * other evaluation on the context invalidates the forward state
 * (DP_E_ARG).  Arguments as for dp_compute. */
int dp_energy(dp_ctx *c, int64_t natoms, const double *coords, const int32_t *types, const double *box,
              double *energy);
int dp_energy_backward(dp_ctx *c, double grad_energy, double *forces, double *virial);

/* Copy the formatted neighbour list of the last evaluation to `nlist`
 * (device, int32 [natoms][sum sel]) and the per-type real counts to `nreal`
 * (device, int32 [natoms][ntypes]); either may be NULL, not both. */
int dp_get_nlist(dp_ctx *c, int32_t *nlist, int32_t *nreal);

/* Copy per-atom intermediates of the last evaluation (device pointers, any
 * may be NULL; layouts as in the oracle):
 *   atom_e [natoms] double; T [natoms][M1][4] double;
 *   D [natoms][M1*M2] double; net_deriv [natoms][sum sel][4] double.
 * The last two are kept only when dp_keep_intermediates(c, 1) was called
 * before the evaluation. */
int dp_keep_intermediates(dp_ctx *c, int keep);
int dp_get_intermediates(dp_ctx *c, double *atom_e, double *T, double *D, double *net_deriv);

int dp_get_stats(dp_ctx *c, dp_stats *out);

/* Velocity-Verlet NVE run (Section VI: the MD loop; 0.5 fs water, 1 fs Cu).
 *   coords, vel [natoms][3] device double (A, A/fs), updated in place;
 *   types [natoms] device int32; box [9] host; masses [ntypes] host amu;
 *   dt in fs; skin in A (candidate list rc+skin, rebuilt when an atom has
 *   moved more than skin/2 since the last build; checked on the device
 *   every step);
 *   thermo: device double [nsteps/thermo_every + 1][6] or NULL, rows
 *   (step, KE, PE, KE+PE, T, P[eV/A^3]), row 0 = the start.
 *   forces [natoms][3] device double or NULL: forces at the final step.
 * The stream is synchronised every thermo_every steps to check flags. */
int dp_md_run(dp_ctx *c, int64_t natoms, double *coords, double *vel, const int32_t *types, const double *box,
              const double *masses, double dt, double skin, int64_t nsteps, int64_t thermo_every,
              double *thermo, double *forces);

/* Per-phase GPU time.  dp_enable_timing(c, 1) starts (or restarts) a record
 * of HIP events on the context's stream around every phase of every
 * evaluation (dp_compute or MD step, at most 2048); dp_get_timing returns
 * the mean milliseconds per evaluation of a phase over that record.
 * names: "lists" (wrap, type order, cells, candidate list), "format"
 * (formatted neighbour list kernel), "env" (environment-matrix kernel),
 * "embed_fwd" (fused embedding + descriptor kernel), "fit" (fitting-net
 * kernels), "embed_bwd" (embedding backward + force/virial kernel),
 * "total" (whole evaluation). */
int dp_enable_timing(dp_ctx *c, int on);
int dp_get_timing(dp_ctx *c, const char *name, double *ms);

const char *dp_last_error(const dp_ctx *c);
void dp_destroy(dp_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* DPMI_H */
