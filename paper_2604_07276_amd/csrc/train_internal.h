// Internal declarations of the student-training kernels (train.hip), used by
// the trainer's host code (train.cpp).  Not part of the public ABI.
//
// Training matches energies and forces (Sec. II-B model, E = sum e_i by
// Eq. (5), F = -dE/dx by Eq. (2)).  With Delta_k = c_f (F_k - F^_k) held
// fixed, the force term's gradient is -d/dtheta of the directional derivative
// E-dot = sum_k Delta_k . dE/dx_k, so one step is: the forward and the force
// adjoint (the inference kernels), a tangent pass along Delta, and a reverse
// sweep of Psi = sum_i (a e_i - e-dot_i) (a = d L_e / dE) back to every weight.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dpa1 {

// Student embedding widths (first, second, third layer): the trainer handles
// the DP-SE-style student 16 -> 32 -> 64 with doubling residuals.
constexpr int kTrN1 = 16, kTrN2 = 32, kTrN3 = 64;

struct TrainPairArgs {
  const float *geom;                 // [P][8] pair records of the inference workspace
  const int *nlist, *nnei, *pair_off;
  const int32_t *types;              // validated types [nall]
  int nloc, sel;
  float inv_sel;
  const float *table;                // [ntypes][ntypes][16] first layer folded with the type embedding
  const float *ws;                   // [16] first-layer weight of s
  const float *W2t, *b2;             // [32][16] (W2 transposed: row o holds W2[:, o]), [32]
  const float *W3t, *b3;             // [64][32], [64]
  int ntypes;
  const float *T;                    // [nloc][4][64] descriptor factor T
  int axis;
};

// Delta_k = cf (F_k - F^_k) as float4; per-block sums of |F - F^|^2 (FP64).
void launch_tr_seed(const double *F, const double *Flab, int n, float cf, float4 *delta,
                    double *sq_part, hipStream_t s);
int tr_seed_blocks(int n);
// a = ca (E - E^), le = cl (E - E^)^2 (one thread).
void launch_tr_energy_seed(const double *E, const double *Elab, double ca, double cl, float *a,
                           double *le, hipStream_t s);
// Tangent pass: T-dot [nloc][4][64] and D-dot rows [nloc][ldD].
void launch_tr_tangent(const TrainPairArgs &a, const float4 *delta, float *Td, float *Xd, int ldD,
                       hipStream_t s);
// Fitting tangent/reverse elementwise steps (two fitting layers of width H,
// identity residual on the second):
//   top: from t2, y2, y1-dot, z2-dot -> [z2-bar; z2-dot-bar] rows and a y2 - y2-dot rows;
//   l0:  from t1, z1-dot, [y1-bar'; y1-dot-bar'] -> [z1-bar; z1-dot-bar].
void launch_tr_fit_top(const float *t2, const float *y2, const float *yd1, const float *zd2,
                       const float *w_out, const float *a, int nloc, int H, int ld, float *zb2,
                       float *wo_rows, hipStream_t s);
void launch_tr_fit_l0(const float *t1, const float *zd1, const float *yb1, const float *w_out,
                      const float *a, int nloc, int H, int ld, float *zb1, hipStream_t s);
// Reverse sweep of the descriptor and the embedding net per pair; writes the
// weight-gradient operands feature-major (feature f of pair row r at
// f * ldr + r; primal rows [0, P), tangent rows [Pcap, Pcap + P)):
//   X3 [32][ldr] = h2 | h2', Z3 [64][ldr] = z3-bar | z3'-bar,
//   X2 [16][ldr] = h1 | h1', Z2 [32][ldr] = z2-bar | z2'-bar,
//   Z1 [16][ldr] = z1-bar, WS1 [16][ldr] = ws-bar per pair (primal rows only),
//   grp [P] = t_j * ntypes + t_i.
// Pcap and ldr are multiples of 16.
// HB2 [64][ldr] is scratch between the two passes (h2-bar | h2'-bar).
void launch_tr_pair_rev(const TrainPairArgs &a, const float4 *delta, const float *Td,
                        const float *Db, int ldD, size_t Pcap, size_t ldr, float *X3, float *Z3,
                        float *X2, float *Z2, float *Z1, float *WS1, float *HB2, int *grp,
                        hipStream_t s);
// As tr_wgrad and tr_colsum for feature-major operands (Xt [kin][ldr], Zt
// [nout][ldr], group [rows]); the second segment starts at row seg2 (0: none).
void tr_wgrad_fm(const float *Xt, const float *Zt, size_t ldr, size_t seg2, int kin, int nout,
                 const int *rows_dev, int rows_max, int bf16, float *part, size_t part_cap,
                 double *acc, hipStream_t s);
void tr_colsum_fm(const float *Zt, size_t ldr, int ncol, const int *rows_dev, int rows_max,
                  const int32_t *group, int ngroups, float *part, size_t part_cap, double *acc,
                  hipStream_t s);
// acc[kin][nout] += sum_r X1[r]^T Z1[r] + X2[r]^T Z2[r] over r < rows (rows
// from *rows_dev when set, else rows_max); FP32 (or BF16-operand) matrix-core
// partials per row block, summed in fixed order in FP64.
void tr_wgrad(const float *X1, const float *X2, int ldx, const float *Z1, const float *Z2, int ldz,
              int kin, int nout, const int *rows_dev, int rows_max, int bf16, float *part,
              size_t part_cap, double *acc, hipStream_t s);
// acc[g][c] += sum over rows r with group[r] == g of Z[r][c] (group == nullptr: g = 0),
// as a matrix-core product with a generated one-hot operand; ngroups <= 64.
void tr_colsum(const float *Z, int ldz, int ncol, const int *rows_dev, int rows_max,
               const int32_t *group, int ngroups, float *part, size_t part_cap, double *acc,
               hipStream_t s);
// Adam on FP32 master weights with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t.
void launch_adam(float *theta, float *m, float *v, const double *g, int n, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t s);
void launch_fill_f64(double *p, size_t n, hipStream_t s);

}  // namespace dpa1

namespace dpa1 {
// Per-block (sum |a - b|^2, max |a_kc - b_kc|) over n atoms of two [n][3] arrays.
int force_error_blocks(int n);
void launch_force_error(const double *a, const double *b, int n, double *part, hipStream_t s);
}  // namespace dpa1
