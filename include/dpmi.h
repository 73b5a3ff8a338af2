/*
 * dpmi.h -- C ABI of the MI355X (gfx950) Deep Potential evaluator.
 *
 * The library computes, for a periodic orthorhombic box of atoms, the Deep
 * Potential energy E = sum_i E_i, the forces F = -dE/dr and the virial
 * Xi = -sum_{i,j} g_ij (x) r_ij, the quantities the paper's MD step spends
 * its time on (Section III, "Deep Potential Molecular Dynamics" and Fig. 1;
 * Section V-B on the neighbour-list format and the custom Environment,
 * ProdForce and ProdVirial operators; Section V-B "Mixed-precision
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
                          per-atom sort buffer (512) holds                  */
};

/* Precision policies (after the paper's MIX-32 and MIX-16 schemes, Section
 * V-B "Mixed-precision computation").
 * DP_FP64: everything in double.
 * DP_MIX_FP32 (the paper's MIX-32): the embedding and fitting nets' weights
 *   rounded to FP32, the environment matrix rounded to FP32, and every
 *   operation of both nets (matrix-core products, tanh, the descriptor
 *   contractions, the backward) in FP32; the per-atom energies and the
 *   network gradient dE/dR are converted to double.  Same net widths as
 *   DP_FP64 (up to 128).
 * DP_MIX_FP16 / DP_MIX_BF16: embedding layers after the first and the first
 *   two fitting layers as 16-bit matrix-core products with FP32
 *   accumulation and 16-bit weights; activations enter those products as
 *   hi + lo 16-bit pairs (about 22 bits); tanh, the descriptor contractions,
 *   the remaining fitting layers and the output layer in FP32.
 * Coordinates, wrapping, distances, the environment matrix (before its
 * rounding), the force Jacobian, energy / force / virial sums and the
 * integrator stay double in every mode. */
enum { DP_FP64 = 0, DP_MIX_FP32 = 1, DP_MIX_BF16 = 2, DP_MIX_FP16 = 3 };

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
  int64_t judge_atoms;       /* atoms the last judge covered                 */
  int64_t cell_scatter;      /* backward passes with the cell-ordered scatter */
  int64_t table_evals;       /* student evaluations with the tabulated layers */
  int64_t wide_evals;        /* evaluations through the wide-net GEMM path */
} dp_stats;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the null stream).  *out receives the context. */
int dp_create(dp_ctx **out, int device, void *hip_stream);

/* Load a model blob (host memory, `nbytes` bytes, layout DPMIBLOB: magic,
 * int64 version/ntypes/n_emb/n_fit/M2, version 2 only: int64 emb_out_linear
 * (1 = the last embedding layer is affine), float64 rcut/rcut_smth/
 * desc_norm, int64 sel[ntypes], emb widths, fit widths, then float64
 * weights) and keep
 * it on the device in `precision` (DP_FP64 ...).  The blob may be freed
 * after the call.  The descriptor is D = T T_<^T with
 * T = (1/desc_norm) sum_j G(s_j) R_j^T (Fig. 1(b)); one embedding net per
 * (centre type, neighbour type) pair and one fitting net per centre type.
 * Embedding widths up to 128 run in every precision; wider nets (up to
 * 2048, the embedding-size study of Sec. VII-D / Fig. 7: hidden widths
 * multiples of 64, later widths multiples of 128, M1 a multiple of 256, at
 * most 4 atom types) run in DP_MIX_FP16 / DP_MIX_BF16 only, as 16-bit GEMMs
 * over all neighbour pairs; DP_FP64 with such a net returns DP_E_MODEL.
 * Their evaluations read the per-net pair counts back to the host once
 * (one synchronisation of the context's stream) to lay out the GEMM rows,
 * and their activation buffers (8 bytes per real pair and feature of the
 * widest layer) are kept until the next dp_set_model or dp_destroy. */
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
 * formatted as in Section V-B (type-sorted, then by distance with ties by
 * index, nearest sel kept per type, -1 padded). */
int dp_compute(dp_ctx *c, int64_t natoms, const double *coords, const int32_t *types, const double *box,
               double *energy, double *forces, double *virial);

/* Rank-share evaluation: the share of one GPU in the spatial domain
 * decomposition of Section V-D ("Reducing MPI communication bottlenecks").
 *   atoms [0, n_local)       the centres this rank owns (a brick of space)
 *   atoms [n_local, natoms)  its ghosts: the atoms (or periodic images)
 *                            within rc of the brick, neighbours only
 * coords, types and box as for dp_compute; no atom may see a periodic image
 * of another within rc unless that image is meant (pad the brick and its
 * shell with rc of vacuum).  Outputs (device, may be NULL):
 *   energy  sum of E_i over the centres
 *   forces  [natoms][3]: -dE_local/dr for every atom, ghosts included; a
 *           ghost's force belongs to the rank owning that atom, which adds
 *           it to its own (dp_scatter_add_forces)
 *   virial  -sum over centres i and their neighbours j of g_ij (x) r_ij, so
 *           the bricks' energies, virials and reverse-added forces sum to
 *           those of the whole system.
 * Every pair force is added with FP64 atomics (no cell-ordered scatter).
 * dp_get_nlist, dp_get_intermediates and dp_energy_backward do not refer to
 * this evaluation.  Wide embedding nets return DP_E_MODEL. */
int dp_compute_local(dp_ctx *c, int64_t n_local, int64_t natoms, const double *coords, const int32_t *types,
                     const double *box, double *energy, double *forces, double *virial);

/* f_out[index[k]][a] += f_in[k][a] for k < n, a < 3 (device arrays; index
 * int32, entries < 0 skipped; FP64 atomics on the context's stream): the
 * reverse communication of a spatial decomposition, adding ghost forces to
 * their owners' (Section V-D). */
int dp_scatter_add_forces(dp_ctx *c, int64_t n, const int32_t *index, const double *f_in, double *f_out);

/* dp_compute without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, results and errors as for dp_compute;
 * the caller still passes coords, types and the outputs.  The workspace is
 * a static device array of 256 MiB, one per GPU, held until the process
 * ends, instead of the context's own: a system whose workspace does not fit
 * it returns DP_E_CAP before any kernel is queued (as a rough guide, for
 * the 1-25-50-100 nets: about 4,600 water or 3,200 copper atoms (sel 138 /
 * 512) in DP_FP64, about 25,000 water or 14,000 copper atoms in
 * DP_MIX_FP16 / DP_MIX_BF16); wide embedding nets (widths above
 * 128) return DP_E_MODEL.  With a student in use whose layer table no
 * dp_compute has built yet, the student's layers are evaluated instead of
 * the table.  The call calls no hipMalloc, hipFree or other allocating
 * routine.  Every call on one GPU, from any context, uses the same array and
 * leaves its contents behind (each call rewrites what it reads): calls that
 * overlap in time on one GPU race and must be serialised by the caller.
 * The context's own workspace, its last lists and a pending dp_energy are
 * left untouched (dp_get_nlist etc. still refer to the last dp_compute). */
int dp_compute_noalloc(dp_ctx *c, int64_t natoms, const double *coords, const int32_t *types, const double *box,
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

/* Neighbour-force scatter of the mixed-precision backward with a student
 * (affine-last-layer) net set; the sums are FP64 either way, only their
 * order differs.
 *   mode 0 (default): cell-ordered -- when the list grid has 3 to 255 cells
 *     per axis, one workgroup per cell accumulates the pair forces on the
 *     27 surrounding cells' atoms in LDS and a gather pass adds the 27
 *     parts of each atom (no global atomics; the LDS holds twice the mean
 *     cell occupancy plus 16 atoms per cell, at most 128, and atoms beyond
 *     that add their forces with atomics); when the nets and that
 *     accumulator do not fit the LDS, as mode 1;
 *   mode 1: every pair force is added to F with FP64 global atomics.
 * Returns DP_E_ARG for another mode. */
int dp_set_force_scatter(dp_ctx *c, int mode);

/* Storage of the per-pair activations of wide embedding nets (widths above
 * 128, the embedding-size study of Sec. VII-D / Fig. 7; see dp_set_model).
 *   mode 0 (default): each activation and tangent as a hi + lo pair of
 *     16-bit values, both multiplied by the 16-bit weights (two products),
 *     as the register-resident kernels do: forces within ~1e-5 relative of
 *     the FP64 evaluation with the same 16-bit weights;
 *   mode 1: one 16-bit value each, the paper's MIX-16 storage (Sec. V-B):
 *     half the products and the activation memory; dE/dR of each pair
 *     within ~2 units of 16-bit roundoff, forces of near-symmetric
 *     structures (small differences of large pair terms) at a few percent.
 * Takes effect from the next evaluation.  Returns DP_E_ARG for another mode. */
int dp_set_wide_storage(dp_ctx *c, int mode);

/* Velocity-Verlet NVE run (Section VI: the MD loop; 0.5 fs water, 1 fs Cu).
 *   coords, vel [natoms][3] device double (A, A/fs), updated in place;
 *   types [natoms] device int32; box [9] host; masses [ntypes] host amu;
 *   dt in fs; skin in A (candidate list rc+skin, rebuilt when an atom has
 *   moved more than skin/2 since the last build; checked on the device
 *   every step);
 *   thermo: device double [nsteps/thermo_every + 1][6] or NULL, rows
 *   (step, KE, PE, KE+PE, T, P[eV/A^3]), row 0 = the start.
 *   forces [natoms][3] device double or NULL: forces at the final step.
 * The stream is synchronised every thermo_every steps (and after the last
 * step) to check the error flags; no other host round trip happens per step.
 * Once a kernel raises an error flag the integrator kernels leave coords and
 * vel as they are, so the run stops on the device at the step where the
 * error arose (coords at that step, vel before its second half kick).  A
 * skin candidate list too small for the local density is then doubled (up
 * to four times per call) and the run resumes at that step, giving the
 * same trajectory as a large enough list from the start; other errors
 * return with coords and vel in that stopped state. */
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
 * kernels and the energy sum), "fit_fwd" / "fit_bwd" (its forward kernel /
 * the energy sum and its backward kernel), "embed_bwd" (embedding backward
 * + force/virial kernel and, with the cell-ordered scatter, the gather
 * pass), "embed_bwd_main" (the embedding backward kernel alone), "total"
 * (whole evaluation). */
int dp_enable_timing(dp_ctx *c, int on);
int dp_get_timing(dp_ctx *c, const char *name, double *ms);

/* ---------------------------------------------------------------------
 * Student embedding net (not in the paper: a smaller stand-in for the
 * embedding nets of Fig. 1(e,f), checked against the full nets while MD
 * runs).  Per (centre type, neighbour type) pair the student is
 * 1 -> 16 (tanh) -> 32 (tanh, doubling skip) -> M1 (affine), and it feeds
 * the teacher's descriptor and fitting net unchanged.  dp_student_train
 * fits it to the teacher's own G(s) on neighbour distances of the last
 * evaluated configuration:
 *   samples  uniform over the real (centre, neighbour) pairs of each type
 *            pair: attempt a of sample q of net n = t*ntypes+u draws
 *            x = SplitMix64 output number ((n*2^40 + q)*32 + a) of the
 *            stream seeded with `seed`; centre = atom number
 *            (x>>32)*count_t>>32 of type t (atoms of a type in index
 *            order), slot = (x & 0xffffffff)*sel_u>>32; kept when the
 *            slot holds a real neighbour (else the next attempt; after 32
 *            the sample has weight 0).  Adam batch k uses q = k*batch ..;
 *            the least squares q = 2^36 + ..; the held-out check q = 2^37 + ..
 *   loss     mean over samples and the M1 outputs of (G_s - G_t)^2, the
 *            teacher's G_t in FP64
 *   Adam     (Kingma and Ba, 2015) in FP32, bias-corrected, constant lr
 *   refit    exact least squares of the affine output layer on the hidden
 *            features (h2, 1): FP64 normal equations + ridge * trace/33 on
 *            the diagonal, Cholesky.  Under DP_MIX_* the W2 used for the
 *            features and the solved W3 are rounded to the 16-bit format of
 *            the kernels, and b3 takes the mean residual.
 * ------------------------------------------------------------------- */
typedef struct {
  int64_t batch;       /* samples per net per Adam step, a multiple of 64 (4096)  */
  int64_t adam_steps;  /* Adam steps (500: 2M samples at batch 4096)               */
  double lr, beta1, beta2, eps; /* 1e-3, 0.9, 0.999, 1e-8                          */
  int64_t ls_samples;  /* samples per net for the refit, multiple of batch (262144) */
  double ridge;        /* relative ridge of the normal equations (1e-14)           */
  uint64_t seed;       /* sampler and initialisation seed                          */
  int32_t init;        /* 1: fresh initialisation; 0: continue from the current
                          parameters (dp_student_set_params or an earlier call)    */
  int32_t refit;       /* 1: least-squares refit and install the student           */
} dp_student_cfg;

/* Fill *cfg with the defaults listed above. */
int dp_student_default_cfg(dp_student_cfg *cfg);

/* Train on the configuration of the last evaluation (dp_compute, dp_energy
 * or the final frame of dp_md_run) and, when cfg->refit, install the
 * student (it is used once dp_student_use(c, 1) is called).
 * fit_rmse (host, may be NULL) receives the relative RMSE of G against the
 * teacher on 4096 held-out samples per net (sqrt(sum err^2 / sum G_t^2),
 * worst net), or the last Adam loss when cfg->refit is 0.  The student's
 * mixed-precision kernels exist for M1 = 100 only (DP_E_MODEL otherwise). */
int dp_student_train(dp_ctx *c, const dp_student_cfg *cfg, double *fit_rmse);

/* FP32 training parameters, [ntypes^2][np] with np = 16+16+16*32+32+32*M1+M1
 * per net laid out W1[16] b1[16] W2[16][32] b2[32] W3[32][M1] b3[M1]
 * (row = input feature); host memory.  set resets the Adam moments. */
int dp_student_get_params(dp_ctx *c, float *params);
int dp_student_set_params(dp_ctx *c, const float *params);

/* Loss and gradient of one Adam batch (`step` = k above, seed as given) at
 * the current parameters, without updating them.  Host outputs, any may be
 * NULL: s [ntypes^2][batch] sampled inputs (0 where the weight is 0),
 * loss [ntypes^2] (mean squared error per net), grad [ntypes^2][np]. */
int dp_student_batch_grad(dp_ctx *c, uint64_t seed, int64_t step, int64_t batch, double *s, double *loss,
                          float *grad);

/* Evaluations (dp_compute, dp_energy, dp_md_run) use the student (on = 1)
 * or the teacher (0).  DP_E_NOMODEL when no student is installed. */
int dp_student_use(dp_ctx *c, int on);

/* MD judge: while the student is in use, dp_md_run also evaluates the
 * teacher every `every` steps (0 = never) on the same configuration and
 * computes the force RMSE sqrt(mean_i |F_s,i - F_t,i|^2); above
 * max_force_rmse (eV/A) the run takes the teacher's forces for that step
 * and uses the teacher for the rest of the run (stats.teacher_fallbacks).
 * Defaults: every 20 steps, 1e-3 eV/A. */
int dp_student_judge(dp_ctx *c, int64_t every, double max_force_rmse);

/* Sampled judge (side > 0, A): the teacher is evaluated only on the atoms of
 * a cube of that side and on the atoms within rc of it, which gives every
 * atom of the cube its exact teacher force; the RMSE of the judge is taken
 * over the cube's atoms.  The cube's centre for the judge at MD step k is
 * L_a * u_a with u_a = (x >> 11) * 2^-53, x = SplitMix64 output number
 * 3k + a of the stream seeded with 0x6a75646765.  A rejected sample is
 * confirmed by a full teacher evaluation before the fallback.  side = 0
 * (the default), or a cube that with its rc margins does not fit the box,
 * judges all atoms. */
int dp_student_judge_sample(dp_ctx *c, double side);

/* The installed student as a model blob (DPMIBLOB version 2: the student
 * embedding nets with an affine last layer, the teacher's fitting nets):
 * writes min(cap, size) bytes to buf (host, may be NULL) and the size to
 * *nbytes.  dp_student_set_model installs a student from such a blob; its
 * ntypes, rcut, rcut_smth, desc_norm, sel, M2 and fitting nets must match
 * the teacher's and its embedding must be 1-16-32-M1 affine. */
int dp_student_get_model(dp_ctx *c, void *buf, size_t cap, size_t *nbytes);

/* Tabulated student layers (mixed precision only; default on).  The first
 * two layers of a student net map the scalar s to h2(s); on the first
 * student evaluation after the student or the precision changes, h2 and
 * dh2/ds are tabulated in FP64 (weights as the 16-bit kernels hold them) on
 * 81 points over [0, 1.25 x the largest s of that frame] and then
 * interpolated by cubic Hermite polynomials per neighbour; a 16-neighbour
 * tile with any s beyond the range evaluates the layers.  on = 0 always
 * evaluates the layers.  The table's own error is far below the student's
 * fitting error (GPU test: forces within 1e-5 eV/A of the evaluated
 * layers). */
int dp_student_table(dp_ctx *c, int on);
int dp_student_set_model(dp_ctx *c, const void *blob, size_t nbytes);

const char *dp_last_error(const dp_ctx *c);
void dp_destroy(dp_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* DPMI_H */
