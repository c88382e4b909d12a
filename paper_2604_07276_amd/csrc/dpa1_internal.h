// Internal declarations shared by the host orchestration and the HIP kernels
// of the DPA-1 library.  Not part of the public ABI (that is include/dpa1.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpa1 {

// ---------------------------------------------------------------------------
// Padded widths.  Activations are stored row-major with a row stride that is
// the width rounded up to 16 (one MFMA k-chunk); the pad columns hold zeros.
// ---------------------------------------------------------------------------
constexpr int kPad = 16;
inline int pad16(int x) { return (x + kPad - 1) / kPad * kPad; }

// tanh x = 1 - 2 / (exp(2x) + 1) with the hardware base-2 exponential and
// reciprocal (v_exp_f32, v_rcp_f32): five VALU operations and no branch.  It
// saturates to +-1 without NaN (exp(2x) = inf gives 1 - 0, exp(2x) = 0 gives
// 1 - 2).  Its error is a few FP32 ulps of 1 in absolute terms (no relative
// accuracy as x -> 0); every activation it feeds is added to O(1) terms or
// enters as 1 - t^2, where that is the rounding level of FP32 storage.
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.88539008177792681f);  // 2 / ln 2
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// Geometry record of one neighbour pair (8 floats):
//   s = sw/r, rhat (3), sw, r, dsw/dr, and the FP32 remainder sw - (float)sw.
enum GeomField { G_S = 0, G_RX = 1, G_RY = 2, G_RZ = 3, G_SW = 4, G_R = 5, G_DSW = 6, G_SWLO = 7 };
constexpr int kGeom = 8;

// Cell grid used for the O(N) neighbour search.
struct CellGrid {
  int periodic;
  int nc[3];
  int ncell;
  double lo[3];        // origin of the grid (0 when periodic)
  double L[3];         // box lengths (periodic only)
  double inv_edge[3];  // cells per Angstrom
};

// Device status flags of one step.
struct DevFlags {
  int overflow_atom;   // smallest atom index with more than sel neighbours, INT_MAX if none
  int overflow_count;  // its neighbour count
  int bad_type_atom;   // smallest atom index with an invalid type, INT_MAX if none
  int pair_overflow;   // the step's pair count when it exceeds the pair arena, else 0
};

// ---------------------------------------------------------------------------
// neighbour search (nlist.hip)
// ---------------------------------------------------------------------------
void launch_check_types(const int32_t *types, int nall, int ntypes, DevFlags *flags,
                        int32_t *safe, hipStream_t s);
void launch_cell_bin(const double *coords, int nall, CellGrid grid, int *atom_cell,
                     int *cell_count, hipStream_t s);
void launch_scan(const int *in, int n, int *out_excl, hipStream_t s);  // out[n] = total
void launch_cell_fill(const int *atom_cell, int nall, const int *cell_start, int *cell_fill,
                      int *cell_atoms, hipStream_t s);
void launch_nlist(const double *coords, int nloc, int nall, CellGrid grid, double rcut,
                  int sel, const int *cell_start, const int *cell_atoms, int *nlist, int *nnei,
                  DevFlags *flags, hipStream_t s);
// Per pair: geometry record and the first embedding layer
// h1 = tanh(type_table[t_j][t_i] + ws * s), 25 -> stride 32.
void launch_env_embed1(const double *coords, const int32_t *types, CellGrid grid, int nloc,
                       int sel, double rcut, double rcut_smth, const int *nlist, const int *nnei,
                       const int *pair_off, const float *type_table, const float *ws, int ntypes,
                       int n1, int ld1, float *geom, float *h1, hipStream_t s);

// ---------------------------------------------------------------------------
// row-batched FP32 MFMA GEMMs with fused epilogues (gemm.hip)
//   Y[M x N] = X[M x K] W[K x N], W passed transposed as Wt[Npad x K].
//   M is read from device memory (*Mptr) when Mptr != nullptr.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const float *X;
  int ldx;
  const float *Wt;
  int K;          // multiple of 16
  int Npad;       // multiple of 16
  int Nreal;
  const int *Mptr;
  int Mmax;       // grid sizing bound
  int bf16;       // 1: BF16 matrix-core operands (FP32 accumulate), 0: FP32
  int xbf16;      // with bf16: X is stored in BF16 (row stride ldx in elements)
  int kreal;      // 0, or the depth up to which X and W hold data (zeros past it)
  int kslice;     // 0, or split k: grid slice z covers depths [z kslice, (z + 1) kslice)
};

enum ResMode { RES_NONE = 0, RES_IDENT = 1, RES_DOUBLE = 2, RES_BCAST = 3, RES_FOLD = 4 };

// y = tanh(acc + b) + res ; optionally also stores the tanh output.
// Per-row bias: bias + row_type[row] * bias_ld when row_type != nullptr.
void gemm_tanh_res(const GemmArgs &a, const float *bias, const int32_t *row_type, int bias_ld,
                   const float *res, int ldr, int res_mode, int res_fin, float *y, int ldy,
                   float *tout, int ldt, hipStream_t s);
// The same product split over k for few rows and a long k (the first fitting
// layer of a small domain): slices of the k range run as separate
// workgroups into partial sums in scratch, one pass adds them in slice
// order and applies the epilogue.  Returns false, launching nothing, when
// the shape does not call for it or scratch (floats) is too small; the
// caller then runs gemm_tanh_res.
bool gemm_tanh_res_split(const GemmArgs &a, const float *bias, const int32_t *row_type,
                         int bias_ld, float *y, int ldy, float *tout, int ldt, float *scratch,
                         size_t scratch_floats, hipStream_t s);
// y = acc + b (b may be null); ybf16: y stored in BF16
void gemm_linear(const GemmArgs &a, const float *bias, float *y, int ldy, hipStream_t s,
                 int ybf16 = 0);
// Attention output projection with layer norm and residual:
//   yv = acc + b; xhat = (yv - mean) * rstd; gout = gin + gamma*xhat + beta.
void gemm_ln_res(const GemmArgs &a, const float *bias, const float *gamma, const float *beta,
                 float eps, const float *gin, int ldg, float *gout, float *xhat, float *rstd,
                 hipStream_t s);
// Backward through a tanh layer: d = acc + res; a = d * (1 - t^2).
void gemm_bwd_tanh(const GemmArgs &a, const float *res, int ldr, int res_mode, int res_fin,
                   const float *t, int ldt, float *d, int ldd, float *aout, int lda,
                   hipStream_t s);
// Backward of the attention input projections:
//   dgin = acc + dgout; then either the layer-norm backward of the previous
//   layer (mode 0: dy = rstd*(gamma*dgin - mean(.) - xhat*mean(gamma*dgin*xhat))),
//   the embedding tanh backward (mode 1: du = dgin * (1 - t^2)) or nothing (mode 2).
void gemm_qkv_bwd(const GemmArgs &a, const float *dgout, int mode, const float *gamma,
                  const float *xhat, const float *rstd, const float *t, float *dgin,
                  float *dnext, hipStream_t s);
// First embedding layer backward: dh1 = acc + residual(dh2) (RES_NONE, RES_IDENT or
// RES_FOLD); du1 = dh1 * (1 - h1^2); gs[row] = sum_o du1[o] * ws[o].
void gemm_emb1_bwd(const GemmArgs &a, const float *dh2, int ldd2, int res_mode, int fin,
                   const float *h1, int ldh1, const float *ws, float *gs, hipStream_t s);

// ---------------------------------------------------------------------------
// fused embedding layers 2..3 and their adjoint (embed.hip)
// ---------------------------------------------------------------------------
struct EmbLaunch {
  const float *h1;        // [P][ld0] first-layer output
  const float *W2t, *b2;  // layer 2, transposed weights [ld1][ld0], bias [ld1]
  const float *W3t, *b3;  // layer 3 [ld2][ld1], [ld2]
  const float *W2b, *W3b; // adjoint operands [ld0][ld1], [ld1][ld2]
  const float *ws;        // first-layer weight of s [ld0]
  int n0, n1, n2;         // real widths
  int res2, res3;         // residual rules (RES_NONE / RES_IDENT / RES_DOUBLE)
  const int *Pptr;        // number of pairs (device)
  int Pmax;
  int bf16;               // 1: BF16 matrix-core operands (FP32 accumulate)
};
bool emb_fused_supported(int ld0, int ld1, int ld2);
void launch_emb_fwd(const EmbLaunch &e, float *G0, hipStream_t s);
// dE/ds per pair from dE/dG0, recomputing the forward of layers 2..3.
void launch_emb_bwd(const EmbLaunch &e, const float *dG0, float *gs, hipStream_t s);

// ---------------------------------------------------------------------------
// per-centre kernels (attn.hip)
// ---------------------------------------------------------------------------
// Gated neighbour self-attention core.  Centres are split by neighbour
// count into classes of 32/64/96/128 slots (class c covers n in
// (32c, 32(c+1)]); every launch below covers one class, over the class's
// centre list, with a persistent grid sized at attn_prepare().
int attn_class_count(int sel);
int attn_class_npad(int cls);
// Row stride of the stored scaled logits (floats per pair).
constexpr int kAttnLamLd = 128;
// Per device, once: LDS limits of the large classes and persistent grid sizes.
hipError_t attn_prepare();
// Class lists from the neighbour counts: ccount [4] (zeroed beforehand),
// clist [4][nloc].
// ccount [8]: centres listed per class [0..3], centres per neighbour-count
// class [4..7]; active: bit set of the classes that are launched (the top
// class of sel always among them).
void launch_attn_classes(const int *nnei, int nloc, int active, int *ccount, int *clist,
                         hipStream_t s);
struct AttnArgs {
  const float *geom;
  const int *pair_off, *nnei, *clist, *ccount;
  int nloc, sel;
  float shift;
  int bf16;  // 1: BF16 matrix-core operands (FP32 accumulate)
  // bit c: class c held no centres in a recent step; its persistent grid is
  // kept to a few blocks (any count is still processed, only more slowly)
  int small = 0;
};
// Output projection and layer norm of an attention layer, applied by the
// forward itself (in BF16 mode with BF16 operands): W_O^T [kAttnOpCols][128]; bias, gamma, beta with
// kAttnOpCols entries (zeros past Nreal); gin, gout, xhat rows of
// kAttnOpCols floats, rstd one per pair.
constexpr int kAttnOpCols = 112;
struct AttnOut {
  const float *Wt_o, *bias, *gamma, *beta;
  float eps;
  const float *gin;
  float *gout, *xhat, *rstd;
  int Nreal;
};
// Forward: O = (P o H) V per centre; stores lam = QK^T/sqrt(d) per pair row
// ([P][kAttnLamLd]) and (m, 1/Z) per pair (fstat, float2).  With op it
// also applies the output projection and layer norm (gout, xhat,
// rstd as the projection GEMM writes them) and stores O only for the
// 128-neighbour class, whose two-kernel adjoint reads it; with op == nullptr
// it stores O for every class.
void launch_attn_fwd_class(int cls, const AttnArgs &a, const float *qkv, float *out, float *lam,
                           float *fstat, const AttnOut *op, hipStream_t s);
// Backward, query tiles: dQ, (m, 1/Z, D_q) and the query-side gate/switch
// gradients (astat, qside: per-pair float4 buffers read by the key-tile pass).
// dA [P][kAttnLamLd]: dL/dA of every (query, key) pair of a centre, in the
// layout of lam, written here and read by the key-tile pass.
void launch_attn_bwd_q_class(int cls, const AttnArgs &a, const float *qkv, const float *o,
                             const float *dO, const float *lam, const float *fstat, float *dqkv,
                             float *astat, float *qside, float *dA, hipStream_t s);
// Backward, key tiles: dK, dV and the total dE/dsw, dE/drhat per pair
// (accumulated onto gw/gr when accumulate != 0).
void launch_attn_bwd_k_class(int cls, const AttnArgs &a, const float *qkv, const float *dO,
                             const float *lam, const float *dA, float *dqkv, const float *astat,
                             const float *qside, float *gw, float *gr, int accumulate,
                             hipStream_t s);
// Both halves of the backward in one kernel (FP32, classes of up to 96
// neighbours; attn_bwd_fused tells whether a class has it): the outputs of
// the query-tile and key-tile passes without dA, astat and qside, and
// without reading O (D_q = sum_k A dA instead of dO . o).
bool attn_bwd_fused(const AttnArgs &a, int cls);
void launch_attn_bwd_fused_class(int cls, const AttnArgs &a, const float *qkv, const float *dO,
                                 const float *lam, const float *fstat, float *dqkv, float *gw,
                                 float *gr, int accumulate, hipStream_t s);
// Descriptor: T = R~^T G / sel (4 x M), D = T^T T[:, :axis] -> dmat [nloc x M*axis].
void launch_desc_fwd(const float *geom, const float *G, int ldg, const int *pair_off,
                     const int *nnei, int nloc, int sel, int M, int axis, float *T, float *dmat,
                     hipStream_t s);
// Descriptor backward and the layer-norm backward of the last attention layer
// (ln_mode 0), the tanh backward of the last embedding layer (1), or dG only (2).
void launch_desc_bwd(const float *geom, const float *G, int ldg, const float *T,
                     const float *dD, const int *pair_off, const int *nnei, int nloc, int sel,
                     int M, int axis, int ln_mode, const float *gamma, const float *xhat,
                     const float *rstd, const float *t_emb, float *dG, float *dnext,
                     float *dRt, hipStream_t s);
// The descriptor adjoint with the layer-norm adjoint of the last attention
// layer (ln_mode 0 above) fused with that layer's output-projection adjoint:
// dG and dR~ as launch_desc_bwd, and dO = d(acc) W_O^T (Wt: [D][ldg], the
// weights the projection adjoint GEMM takes) written in place of d(acc)
// (FP32, or BF16 with bf16).  Shapes: desc_oproj_fusable.
bool desc_oproj_fusable(int ldg, int M, int axis, int D);
void launch_desc_oproj_bwd(const float *geom, const float *G, const float *T, const float *dD,
                           const int *pair_off, const int *nnei, int nloc, int sel, int M,
                           int axis, const float *gamma, const float *xhat, const float *rstd,
                           const float *Wt, float *dG, float *dRt, float *dO, int bf16,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// energies, pair gradients, forces, virial (misc.hip)
// ---------------------------------------------------------------------------
// e_i = z3 . w_out + b_out + ebias[type_i]; a3 = w_out * (1 - t3^2).
void launch_energy(const float *z3, const float *t3, int ld, int nfit, const float *w_out,
                   float b_out, const float *ebias, const int32_t *types, int nloc, float *e,
                   float *a3, hipStream_t s);
// g_ij = de_i/dd_ij from the per-pair upstream gradients.
void launch_env_bwd(const float *geom, const float *gs, const float *dRt, const float *gw,
                    const float *gr, const int *Mptr, int Mmax, float sel_inv_unused,
                    float *g, hipStream_t s);
// Forces by a deterministic gather over the full neighbour lists, per-centre
// virial partials and FP64 outputs.  With per-centre weights wgt (nullable =
// all ones) the result is sign * (-sum_i wgt_i de_i/dx_k); sign = +1 gives
// forces, sign = -1 the gradient of sum_i wgt_i e_i.
void launch_forces(const double *coords, CellGrid grid, int nloc, int nall, int sel,
                   const int *nlist, const int *nnei, const int *pair_off, const float *g,
                   const double *wgt, double sign, double *forces, double *vir_part,
                   hipStream_t s);
// E = sum e_i, Xi = sum of partials (fixed-order FP64 reductions); atom_energy.
// energy == nullptr skips the energy part, virial == nullptr the virial part.
void launch_reduce(const float *e, const double *vir_part, int nloc, double *energy,
                   double *virial, double *atom_energy, hipStream_t s);

}  // namespace dpa1
