/*
 * dpa1.h - C ABI of the MI355X DPA-1 inference library.
 *
 * One call evaluates a DPA-1 deep potential for one MD step on one domain:
 * the energy of the local atoms, the forces on local and ghost atoms and the
 * virial.  This mirrors the per-step inference call of a DeePMD-style model
 * inside a domain-decomposed MD engine: the caller flags which atoms are
 * local and which are ghosts, energies are summed over local atoms only and
 * ghost forces are returned for the caller to reduce onto their owners
 * (Sec. II-C, Eq. (7)).  The library is not MPI-aware; it sees one domain.
 *
 * Units: Angstrom and eV.  Arrays are row-major, atoms are ordered locals
 * first, then ghosts: atom k is local iff k < nloc.
 *
 * Model: energy E = sum_{i<nloc} e_i with e_i = Phi(D^i) (Sec. II-B and
 * Eq. (5)); descriptor D^i = G^T R~ R~^T G_< over the full neighbour list
 * of i within rcut (Sec. II-B; Sec. II-C full lists); G from a type-embedded
 * embedding net refined by gated self-attention inside the neighbour set
 * (Sec. II-B, DPA-1); forces F = -dE/dx (Eq. (2)).
 *
 * Precision: neighbour search and minimum-image pair vectors in FP64; the
 * network in FP32 (FP32 MFMA); energy, force and virial reductions in FP64.
 * Results are deterministic: the same inputs give bit-identical outputs.
 *
 * Ownership: the caller owns every array it passes.  A dp_model owns its
 * device weights and workspace.  A handle is not thread-safe and must not be
 * used by two calls at once (one handle per stream).
 *
 * Errors: every function returns DP_OK (0) or a negative dp_status;
 * dp_last_error() gives a message for the calling thread.  Argument checks
 * run before any device work; on error no output is written.
 */
#ifndef DPA1_H
#define DPA1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_model dp_model;

enum dp_status {
  DP_OK = 0,
  DP_ERR_ARG = -1,           /* NULL pointer, negative count, rcut/sel out of range */
  DP_ERR_TYPE = -2,          /* atom type outside [0, ntypes) */
  DP_ERR_BOX = -3,           /* non-orthorhombic box or a box length <= 2 rcut */
  DP_ERR_SEL_OVERFLOW = -4,  /* an atom has more than sel neighbours within rcut */
  DP_ERR_WEIGHTS = -5,       /* weights file missing, malformed or unsupported */
  DP_ERR_DEVICE = -6,        /* HIP runtime error */
  DP_ERR_OOM = -7,           /* device allocation failed, or the memory budget is too small */
  DP_ERR_CAPACITY = -8       /* a device-memory step had more neighbour pairs than its
                                workspace holds: its outputs are not valid; the workspace is
                                laid out for the larger count at the next call */
};

/* Largest supported neighbour capacity. */
#define DP_MAX_SEL 128

/*
 * Load a weights file and upload the model to the current HIP device: the
 * DPA-1 model of Sec. II-B (type embedding, embedding net, gated attention
 * layers, fitting net) with the cutoff rcut of the neighbour lists (Sec. II-C).
 *   weights_path  file in the DPA-1 weights format (magic "DPA1WTS"), FP64
 *                 tensors; they are rounded to FP32 once here.
 *   rcut          cutoff radius in Angstrom, > rcut_smth of the file.
 *   sel           neighbour capacity, 1 <= sel <= DP_MAX_SEL.  It also sets
 *                 the attention normalisation, which adds (sel - n_i) e^{-S}
 *                 so that energies stay smooth when a neighbour crosses rcut.
 *   out           receives the handle; release with dp_destroy.
 */
int dp_create(const char *weights_path, double rcut, int sel, dp_model **out);

/*
 * Host-memory step (the per-step inference call of Sec. II-C: energy of the
 * local atoms, forces on locals and ghosts per Eq. (7), F = -dE/dx per
 * Eq. (2), one result copy back per output): copies inputs to the device,
 * runs the step on the handle's own stream, copies results back and waits.
 *   coords       [(nloc+nghost)*3] FP64 positions.
 *   types        [nloc+nghost], each in [0, ntypes).
 *   box          [9] FP64, rows are the cell vectors (orthorhombic only, each
 *                length > 2 rcut; minimum image is applied to every pair), or
 *                NULL for open boundaries (the caller supplies image ghosts).
 *   nloc, nghost counts, >= 0.
 *   energy       out: sum of e_i over local atoms.
 *   forces       out: [(nloc+nghost)*3]; ghost atoms receive
 *                -sum_{i local} de_i/dx_ghost (Eq. (7)).
 *   virial       out: [9], Xi_ab = -sum_{i<nloc} sum_j d_ij,a de_i/dd_ij,b
 *                with d_ij = x_j - x_i (equals sum_k x_k,a F_k,b when open).
 *   atom_energy  optional out [nloc] (e_i), or NULL.
 * Returns DP_ERR_SEL_OVERFLOW when some atom (local, or ghost counting its
 * local neighbours) has more than sel neighbours; nothing is written then.
 */
int dp_compute(dp_model *m, const double *coords, const int32_t *types, const double *box,
               int nloc, int nghost, double *energy, double *forces, double *virial,
               double *atom_energy);

/*
 * Device-memory step (the same computation as dp_compute: Sec. II-C,
 * Eq. (2), Eq. (7)), asynchronous on the caller's stream (hipStream_t, NULL
 * for the default stream).  d_coords, d_types, d_energy [1], d_forces, d_virial
 * [9] and d_atom_energy (optional) are device pointers with the layouts of
 * dp_compute; box is a host pointer as above.  The call returns after
 * enqueueing, except in two cases where it first waits on the stream: with
 * box == NULL (open boundaries) it reads the atoms' bounding box back to size
 * the cell grid, and at the first step of a workspace (or after it grew) it
 * reads the step's neighbour-pair count back to lay out the per-pair buffers.
 * Conditions found on the device (an out-of-range type, a neighbour overflow,
 * more neighbour pairs than the workspace holds: DP_ERR_CAPACITY) are
 * reported by dp_sync, and the outputs of such a step are not meaningful.
 */
int dp_compute_device(dp_model *m, const double *d_coords, const int32_t *d_types,
                      const double *box, int nloc, int nghost, double *d_energy,
                      double *d_forces, double *d_virial, double *d_atom_energy,
                      void *hip_stream);

/*
 * Forward half of dp_compute_device, for use under reverse-mode automatic
 * differentiation: computes d_energy [1] and (optionally) d_atom_energy
 * [nloc] on the caller's stream and keeps every activation the adjoint needs
 * in the handle.  The coordinates at d_coords must stay unchanged until the
 * matching dp_backward_device has been enqueued.  Forces are the negative
 * gradient of the energy (Eq. (2)); splitting the step this way lets a caller
 * put per-atom weights on the energies (Eq. (5): E = sum e_i).
 */
int dp_forward_device(dp_model *m, const double *d_coords, const int32_t *d_types,
                      const double *box, int nloc, int nghost, double *d_energy,
                      double *d_atom_energy, void *hip_stream);

/*
 * Adjoint of the last dp_forward_device on this handle: writes
 * d_grad_coords [(nloc+nghost)*3] = d(sum_i w_i e_i)/dx for every atom
 * (ghosts included, Eq. (7)), with w = d_atom_weight [nloc] (device, or NULL
 * for all ones), and optionally the weighted virial d_virial [9]
 * (Xi_ab = -sum_i w_i sum_j d_ij,a de_i/dd_ij,b).  May be called more than
 * once per forward with different weights.  Asynchronous on the stream.
 */
int dp_backward_device(dp_model *m, const double *d_atom_weight, double *d_grad_coords,
                       double *d_virial, void *hip_stream);

/* Precision of the matrix-core products.  The paper's model runs in FP32
 * only (Sec. IV-B); the BF16 mode is an extension of this library.
 *   DP_PREC_FP32  FP32 operands (default).
 *   DP_PREC_BF16  every product of the embedding net, the attention blocks
 *                 (Q K^T, A V, projections and their adjoints) and the
 *                 fitting net takes BF16 operands rounded to nearest even,
 *                 with FP32 accumulation; geometry, switch, descriptor,
 *                 softmax, layer norms and activations stay FP32, energy,
 *                 force and virial reductions FP64.
 * Applies to the steps enqueued after the call; waits for the handle's last
 * step.  Returns DP_ERR_ARG for any other value. */
enum dp_precision { DP_PREC_FP32 = 0, DP_PREC_BF16 = 1 };
int dp_set_precision(dp_model *m, int precision);

/* Memory budget of the workspace in bytes (0: unlimited, the default); the
 * motive is the memory growth of DP inference with system size (Sec. VI-B:
 * ~7 GB for a small protein, an estimated >200 GB for 15k atoms).  The
 * workspace holds its per-pair buffers for the real neighbour-pair count of
 * the step that laid it out plus 1/8, not for nloc * sel pairs.  When
 * storing the activations of every attention layer for the adjoint would make
 * the workspace exceed it, the attention layers share one set of QKV,
 * attention-output, logit and softmax-statistics buffers and the adjoint
 * recomputes each earlier layer's forward from its stored input just before
 * that layer's backward: the results are bit-identical, at the cost of about
 * one attention forward per extra layer.  A step whose workspace exceeds the
 * budget even so returns DP_ERR_OOM.  Takes effect at the next step (the
 * workspace is released and laid out again); waits for the handle's last
 * step.  Returns DP_ERR_ARG for a negative or non-finite budget. */
int dp_set_memory_budget(dp_model *m, double bytes);

/* Workspace bytes currently allocated (per-atom, per-centre and per-pair
 * buffers) and whether the attention activations are recomputed in the
 * adjoint (1) or stored per layer (0). */
int dp_memory_info(const dp_model *m, int64_t *workspace_bytes, int32_t *recompute);

/* Wait for the handle's last step and return its device-side status
 * (DP_ERR_TYPE, DP_ERR_SEL_OVERFLOW or DP_ERR_CAPACITY found on the device).
 * Library plumbing: no passage of the paper defines it. */
int dp_sync(dp_model *m);

/*
 * Neighbour list of the last completed step (the full list within rcut of
 * Sec. II-C, locals and ghosts as neighbours): nlist [nloc*sel] with the
 * neighbours of local atom i in ascending index order, padded with -1, and
 * nnei [nloc].  Host pointers; waits for the step.
 */
int dp_debug_nlist(dp_model *m, int32_t *nlist, int32_t *nnei);

/*
 * Per-kernel timing (measurement plumbing; no passage of the paper defines
 * it).  When enabled, every launch of a step is bracketed by HIP events on
 * its stream.  dp_kernel_times fills, for up to max entries,
 * the kernel name (NUL-terminated, 48 bytes each), the launch count and the
 * summed duration in milliseconds since the last reset; it returns the number
 * of distinct kernels.
 */
int dp_set_timing(dp_model *m, int enable);
int dp_kernel_times(dp_model *m, char *names, int64_t *counts, double *total_ms, int max);

/* Model hyper-parameters of the loaded DPA-1 model (Sec. II-B):
 * ints[8] = ntypes, tebd_dim, axis, n_attn, attn_dim,
 * embedding width M, fitting width, sel; dbls[3] = rcut, rcut_smth, attn_shift. */
int dp_model_info(const dp_model *m, int32_t *ints, double *dbls);

/* Release a handle: waits for its last step, frees its device weights and
 * workspace.  NULL is ignored.  Library plumbing (no passage of the paper
 * defines it). */
void dp_destroy(dp_model *m);

/* Message for the last nonzero return on the calling thread ("" if none).
 * Library plumbing (no passage of the paper defines it). */
const char *dp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DPA1_H */
