// Host side of the student trainer (include/dpa1_train.h).
//
// One batch, per frame: the inference kernels give the student's energy,
// forces and every forward activation; the seeds set Delta = c_f (F - F^) and
// a = c_a (E - E^); the tangent pass gives T-dot and D-dot; the fitting net
// is swept backwards through its values and tangents (matrix-core GEMMs of
// the inference library plus elementwise kernels); the pair kernel sweeps the
// descriptor and the embedding net backwards; the weight gradients are summed
// in FP64 on the device.  After the batch the per-layer sums are chained on
// the host through the folded first layers (type table, per-type fitting
// bias) into weights-file order, Adam updates the FP32 masters on the device,
// and the inference weights are refreshed from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dpa1.h"
#include "dpa1_internal.h"
#include "dpa1_model.h"
#include "dpa1_train.h"
#include "train_internal.h"

using namespace dpa1;

struct dp_trainer {
  dp_model *m = nullptr;
  dp_train_options opt{};
  // weights-file image: header bytes, then the tensors (FP64) in file order
  std::vector<char> header;
  std::vector<std::string> names;
  std::vector<size_t> offs;
  int nparams = 0;
  std::vector<float> theta_h;  // host copy of the masters
  float *theta = nullptr, *am = nullptr, *av = nullptr;
  double *grad_d = nullptr;
  int adam_t = 0;
  // accumulators (FP64) of the per-layer sums, one block
  double *acc = nullptr;
  size_t acc_n = 0;
  size_t o_W2 = 0, o_b2 = 0, o_W3 = 0, o_b3 = 0, o_tab = 0, o_ws = 0, o_W0d = 0, o_fb0 = 0,
         o_W1f = 0, o_b1f = 0, o_wout = 0;
  // capacity-sized buffers
  void *arena = nullptr;
  int cap_n = 0, cap_frames = 0;
  size_t Pcap = 0, ldr = 0;
  double *Fst = nullptr, *Est = nullptr, *vir = nullptr, *sq_part = nullptr, *le = nullptr;
  float *a_dev = nullptr;
  float4 *delta = nullptr;
  float *Td = nullptr, *Xd = nullptr, *Zd1 = nullptr, *Yd1 = nullptr, *Zd2 = nullptr,
        *WoR = nullptr, *Zb2 = nullptr, *Yb1 = nullptr, *Zb1 = nullptr, *Db = nullptr;
  float *X3 = nullptr, *Z3 = nullptr, *X2 = nullptr, *Z2 = nullptr, *Z1 = nullptr,
        *WS1 = nullptr, *HB2 = nullptr;
  int *grp = nullptr;
  float *part = nullptr;
  size_t part_cap = 0;

  ~dp_trainer() {
    if (arena) (void)hipFree(arena);
    if (theta) (void)hipFree(theta);
    if (am) (void)hipFree(am);
    if (av) (void)hipFree(av);
    if (grad_d) (void)hipFree(grad_d);
    if (acc) (void)hipFree(acc);
    if (m) dp_destroy(m);
  }
};

namespace {

size_t param_offset(const dp_trainer *t, const char *name) {
  for (size_t k = 0; k < t->names.size(); ++k)
    if (t->names[k] == name) return t->offs[k];
  return (size_t)-1;
}

// Tensor list of an attention-free model in file order (the weights format).
void tensor_list(const dp_model *m, dp_trainer *t) {
  auto add = [&](const std::string &n, size_t cnt) {
    t->names.push_back(n);
    t->offs.push_back(t->nparams);
    t->nparams += (int)cnt;
  };
  const int T = m->ntypes, E = m->tebd;
  add("type_embedding", (size_t)T * E);
  int fin = 1 + 2 * E;
  for (size_t l = 0; l < m->emb.size(); ++l) {
    add("emb" + std::to_string(l) + ".W", (size_t)fin * m->emb[l]);
    add("emb" + std::to_string(l) + ".b", m->emb[l]);
    fin = m->emb[l];
  }
  fin = m->M * m->axis + E;
  for (size_t l = 0; l < m->fit.size(); ++l) {
    add("fit" + std::to_string(l) + ".W", (size_t)fin * m->fit[l]);
    add("fit" + std::to_string(l) + ".b", m->fit[l]);
    fin = m->fit[l];
  }
  add("w_out", fin);
  add("b_out", 1);
  add("energy_bias", T);
}

std::vector<char> make_image(const dp_trainer *t) {
  std::vector<char> img(t->header);
  const size_t h = img.size();
  img.resize(h + sizeof(double) * t->nparams);
  for (int k = 0; k < t->nparams; ++k) {
    const double v = (double)t->theta_h[k];
    memcpy(img.data() + h + sizeof(double) * k, &v, sizeof(double));
  }
  return img;
}

int ensure_buffers(dp_trainer *t, int n, int nframes) {
  if (n <= t->cap_n && nframes <= t->cap_frames) return DP_OK;
  const int cn = std::max(n, t->cap_n), cf = std::max(nframes, t->cap_frames);
  dp_model *m = t->m;
  const size_t P = ((size_t)cn * m->sel + 15) / 16 * 16;
  // feature-major pair operands: primal rows [0, P), tangent rows [P, 2 P), and one
  // 16-row step of slack read (masked) past the last row
  const size_t ldr = 2 * P + 16;
  const int ldD = m->ldD, ldf0 = m->ldf[0], ldf1 = m->ldf[1];
  const int nsq = tr_seed_blocks(cn);
  // per-centre GEMM operands keep one 16-row tile of slack
  const size_t r1 = (size_t)cn + 16, r2 = 2 * (size_t)cn + 16;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  };
  const size_t oF = take(sizeof(double) * 3 * cn), oE = take(sizeof(double) * cf),
               oV = take(sizeof(double) * 9), oSq = take(sizeof(double) * nsq * cf),
               oLe = take(sizeof(double) * cf), oA = take(sizeof(float) * cf),
               oDelta = take(sizeof(float4) * cn), oTd = take(sizeof(float) * cn * 4 * kTrN3),
               oXd = take(sizeof(float) * r1 * ldD), oZd1 = take(sizeof(float) * r1 * ldf0),
               oYd1 = take(sizeof(float) * r1 * ldf0), oZd2 = take(sizeof(float) * r1 * ldf1),
               oWoR = take(sizeof(float) * r1 * ldf1), oZb2 = take(sizeof(float) * r2 * ldf1),
               oYb1 = take(sizeof(float) * r2 * ldf0), oZb1 = take(sizeof(float) * r2 * ldf0),
               oDb = take(sizeof(float) * r2 * ldD),
               oX3 = take(sizeof(float) * ldr * kTrN2), oZ3 = take(sizeof(float) * ldr * kTrN3),
               oX2 = take(sizeof(float) * ldr * kTrN1), oZ2 = take(sizeof(float) * ldr * kTrN2),
               oZ1 = take(sizeof(float) * ldr * kTrN1), oWS1 = take(sizeof(float) * ldr * kTrN1),
               oHB2 = take(sizeof(float) * ldr * kTrN2), oGrp = take(sizeof(int) * (P + 16));
  if (ldr * kTrN3 >= ((size_t)1 << 32))
    return fail(DP_ERR_ARG, "natoms * sel = %zu pair rows exceed the trainer's limit", P);
  const size_t part_cap = (size_t)1 << 22;
  const size_t oPart = take(sizeof(float) * part_cap);
  if (t->arena) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(t->arena));
    t->arena = nullptr;
  }
  HIP_TRY(hipMalloc(&t->arena, off));
  HIP_TRY(hipMemset(t->arena, 0, off));
  char *b = (char *)t->arena;
  t->Fst = (double *)(b + oF);
  t->Est = (double *)(b + oE);
  t->vir = (double *)(b + oV);
  t->sq_part = (double *)(b + oSq);
  t->le = (double *)(b + oLe);
  t->a_dev = (float *)(b + oA);
  t->delta = (float4 *)(b + oDelta);
  t->Td = (float *)(b + oTd);
  t->Xd = (float *)(b + oXd);
  t->Zd1 = (float *)(b + oZd1);
  t->Yd1 = (float *)(b + oYd1);
  t->Zd2 = (float *)(b + oZd2);
  t->WoR = (float *)(b + oWoR);
  t->Zb2 = (float *)(b + oZb2);
  t->Yb1 = (float *)(b + oYb1);
  t->Zb1 = (float *)(b + oZb1);
  t->Db = (float *)(b + oDb);
  t->X3 = (float *)(b + oX3);
  t->Z3 = (float *)(b + oZ3);
  t->X2 = (float *)(b + oX2);
  t->Z2 = (float *)(b + oZ2);
  t->Z1 = (float *)(b + oZ1);
  t->WS1 = (float *)(b + oWS1);
  t->HB2 = (float *)(b + oHB2);
  t->grp = (int *)(b + oGrp);
  t->part = (float *)(b + oPart);
  t->part_cap = part_cap;
  t->Pcap = P;
  t->ldr = ldr;
  t->cap_n = cn;
  t->cap_frames = cf;
  return DP_OK;
}

// Loss and the FP64 gradient in file order (host) at the current weights.
int batch_gradient(dp_trainer *t, const double *d_frames, const int32_t *d_types,
                   const double *box, int N, int B, const double *d_e_label,
                   const double *d_f_label, double *loss, std::vector<double> &grad,
                   hipStream_t s) {
  dp_model *m = t->m;
  int rc;
  if ((rc = ensure_buffers(t, N, B))) return rc;
  const int ldD = m->ldD, ldf0 = m->ldf[0], ldf1 = m->ldf[1];
  const int H0 = m->fit[0], H1 = m->fit[1], T = m->ntypes;
  const double pe = t->opt.pref_e, pf = t->opt.pref_f;
  const float cf = (float)(2.0 * pf / (3.0 * N * B));
  const double ca = 2.0 * pe / ((double)N * N * B), cl = pe / ((double)N * N * B);
  const int nsq = tr_seed_blocks(N);
  // pair-row stride of the feature-major operands: the tangent rows start at Pst
  const size_t Pst = ((size_t)N * m->sel + 15) / 16 * 16;
  launch_fill_f64(t->acc, t->acc_n, s);
  for (int f = 0; f < B; ++f) {
    const double *xf = d_frames + (size_t)3 * N * f;
    if ((rc = dp_compute_device(m, xf, d_types, box, N, 0, t->Est + f, t->Fst, t->vir, nullptr,
                                s)))
      return rc;
    rc = dp_sync(m);
    if (rc == DP_ERR_CAPACITY) {  // the frame outgrew the pair arena: again on the grown one
      if ((rc = dp_compute_device(m, xf, d_types, box, N, 0, t->Est + f, t->Fst, t->vir,
                                  nullptr, s)))
        return rc;
      rc = dp_sync(m);
    }
    if (rc) return rc;
    auto &w = m->w;
    launch_tr_seed(t->Fst, d_f_label + (size_t)3 * N * f, N, cf, t->delta,
                   t->sq_part + (size_t)nsq * f, s);
    launch_tr_energy_seed(t->Est + f, d_e_label + f, ca, cl, t->a_dev + f, t->le + f, s);
    TrainPairArgs pa{};
    pa.geom = w.geom;
    pa.nlist = w.nlist;
    pa.nnei = w.nnei;
    pa.pair_off = w.pair_off;
    pa.types = w.types_safe;
    pa.nloc = N;
    pa.sel = m->sel;
    pa.inv_sel = 1.0f / (float)m->sel;
    pa.table = m->type_table;
    pa.ws = m->ws;
    pa.W2t = m->embl[1].Wt;
    pa.b2 = m->embl[1].b;
    pa.W3t = m->embl[2].Wt;
    pa.b3 = m->embl[2].b;
    pa.ntypes = T;
    pa.T = w.T;
    pa.axis = m->axis;
    launch_tr_tangent(pa, t->delta, t->Td, t->Xd, ldD, s);
    // fitting net: tangents forward, then values and tangents backward
    const Linear &L0 = m->fitl[0], &L1 = m->fitl[1];
    const int bf = m->bf16;
    gemm_bwd_tanh(GemmArgs{t->Xd, ldD, L0.Wt, ldD, ldf0, H0, nullptr, N, bf}, nullptr, 0,
                  RES_NONE, 0, w.tf[0], ldf0, t->Zd1, ldf0, t->Yd1, ldf0, s);
    gemm_linear(GemmArgs{t->Yd1, ldf0, L1.Wt, ldf0, ldf1, H1, nullptr, N, bf}, nullptr, t->Zd2,
                ldf1, s);
    launch_tr_fit_top(w.tf[1], w.z[1], t->Yd1, t->Zd2, m->w_out, t->a_dev + f, N, H1, ldf1,
                      t->Zb2, t->WoR, s);
    gemm_linear(GemmArgs{t->Zb2, ldf1, L1.Wb, ldf1, ldf0, H0, nullptr, 2 * N, bf}, nullptr,
                t->Yb1, ldf0, s);
    launch_tr_fit_l0(w.tf[0], t->Zd1, t->Yb1, m->w_out, t->a_dev + f, N, H0, ldf0, t->Zb1, s);
    gemm_linear(GemmArgs{t->Zb1, ldf0, L0.Wb, ldf0, ldD, m->M * m->axis, nullptr, 2 * N, bf},
                nullptr, t->Db, ldD, s);
    // descriptor and embedding net
    const size_t ldr = t->ldr;
    launch_tr_pair_rev(pa, t->delta, t->Td, t->Db, ldD, Pst, ldr, t->X3, t->Z3, t->X2, t->Z2,
                       t->Z1, t->WS1, t->HB2, t->grp, s);
    const int *Pdev = w.pair_off + N;
    const int Pmax = (int)Pst;
    tr_wgrad_fm(t->X3, t->Z3, ldr, Pst, kTrN2, kTrN3, Pdev, Pmax, bf, t->part, t->part_cap,
                t->acc + t->o_W3, s);
    tr_wgrad_fm(t->X2, t->Z2, ldr, Pst, kTrN1, kTrN2, Pdev, Pmax, bf, t->part, t->part_cap,
                t->acc + t->o_W2, s);
    tr_colsum_fm(t->Z3, ldr, kTrN3, Pdev, Pmax, nullptr, 1, t->part, t->part_cap,
                 t->acc + t->o_b3, s);
    tr_colsum_fm(t->Z2, ldr, kTrN2, Pdev, Pmax, nullptr, 1, t->part, t->part_cap,
                 t->acc + t->o_b2, s);
    tr_colsum_fm(t->Z1, ldr, kTrN1, Pdev, Pmax, t->grp, T * T, t->part, t->part_cap,
                 t->acc + t->o_tab, s);
    tr_colsum_fm(t->WS1, ldr, kTrN1, Pdev, Pmax, nullptr, 1, t->part, t->part_cap,
                 t->acc + t->o_ws, s);
    tr_wgrad(w.z[0], t->Yd1, ldf0, t->Zb2, t->Zb2 + (size_t)N * ldf1, ldf1, H0, H1, nullptr, N,
             bf, t->part, t->part_cap, t->acc + t->o_W1f, s);
    tr_colsum(t->Zb2, ldf1, H1, nullptr, N, nullptr, 1, t->part, t->part_cap, t->acc + t->o_b1f,
              s);
    tr_wgrad(w.dmat, t->Xd, ldD, t->Zb1, t->Zb1 + (size_t)N * ldf0, ldf0, m->M * m->axis, H0,
             nullptr, N, bf, t->part, t->part_cap, t->acc + t->o_W0d, s);
    tr_colsum(t->Zb1, ldf0, H0, nullptr, N, w.types_safe, T, t->part, t->part_cap,
              t->acc + t->o_fb0, s);
    tr_colsum(t->WoR, ldf1, H1, nullptr, N, nullptr, 1, t->part, t->part_cap, t->acc + t->o_wout,
              s);
    HIP_TRY(hipGetLastError());
  }
  // results to the host
  std::vector<double> acc(t->acc_n), sq((size_t)nsq * B), le(B);
  std::vector<float> av(B);
  std::vector<int32_t> types(N);
  HIP_TRY(hipMemcpyAsync(acc.data(), t->acc, sizeof(double) * t->acc_n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(sq.data(), t->sq_part, sizeof(double) * sq.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(le.data(), t->le, sizeof(double) * B, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(av.data(), t->a_dev, sizeof(float) * B, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(types.data(), m->w.types_safe, sizeof(int32_t) * N,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double lsum_e = 0.0, sqsum = 0.0;
  for (int f = 0; f < B; ++f) lsum_e += le[f];
  for (double v : sq) sqsum += v;
  const double lsum_f = pf / (3.0 * N * B) * sqsum;
  loss[0] = lsum_e + lsum_f;
  loss[1] = lsum_e;
  loss[2] = lsum_f;

  // chain the per-layer sums into file order
  grad.assign(t->nparams, 0.0);
  const int E = m->tebd, n1 = m->emb[0], nd = m->M * m->axis;
  const float *th = t->theta_h.data();
  const size_t pT = param_offset(t, "type_embedding"), pW0 = param_offset(t, "emb0.W"),
               pb0 = param_offset(t, "emb0.b"), pW1 = param_offset(t, "emb1.W"),
               pb1 = param_offset(t, "emb1.b"), pW2 = param_offset(t, "emb2.W"),
               pb2 = param_offset(t, "emb2.b"), pF0 = param_offset(t, "fit0.W"),
               pfb0 = param_offset(t, "fit0.b"), pF1 = param_offset(t, "fit1.W"),
               pfb1 = param_offset(t, "fit1.b"), pwo = param_offset(t, "w_out"),
               pbo = param_offset(t, "b_out"), peb = param_offset(t, "energy_bias");
  const double *tab = acc.data() + t->o_tab;  // [tj][ti][n1]
  for (int o = 0; o < n1; ++o) grad[pW0 + o] = acc[t->o_ws + o];
  for (int a = 0; a < T; ++a)
    for (int b = 0; b < T; ++b)
      for (int o = 0; o < n1; ++o) {
        const double g = tab[((size_t)a * T + b) * n1 + o];
        grad[pb0 + o] += g;
        for (int k = 0; k < E; ++k) {
          grad[pW0 + (size_t)(1 + k) * n1 + o] += g * th[pT + (size_t)a * E + k];
          grad[pW0 + (size_t)(1 + E + k) * n1 + o] += g * th[pT + (size_t)b * E + k];
          grad[pT + (size_t)a * E + k] += g * th[pW0 + (size_t)(1 + k) * n1 + o];
          grad[pT + (size_t)b * E + k] += g * th[pW0 + (size_t)(1 + E + k) * n1 + o];
        }
      }
  for (size_t k = 0; k < (size_t)kTrN1 * kTrN2; ++k) grad[pW1 + k] = acc[t->o_W2 + k];
  for (int k = 0; k < kTrN2; ++k) grad[pb1 + k] = acc[t->o_b2 + k];
  for (size_t k = 0; k < (size_t)kTrN2 * kTrN3; ++k) grad[pW2 + k] = acc[t->o_W3 + k];
  for (int k = 0; k < kTrN3; ++k) grad[pb2 + k] = acc[t->o_b3 + k];
  for (size_t k = 0; k < (size_t)nd * H0; ++k) grad[pF0 + k] = acc[t->o_W0d + k];
  for (int a = 0; a < T; ++a)
    for (int o = 0; o < H0; ++o) {
      const double g = acc[t->o_fb0 + (size_t)a * H0 + o];
      grad[pfb0 + o] += g;
      for (int k = 0; k < E; ++k) {
        grad[pF0 + (size_t)(nd + k) * H0 + o] += g * th[pT + (size_t)a * E + k];
        grad[pT + (size_t)a * E + k] += g * th[pF0 + (size_t)(nd + k) * H0 + o];
      }
    }
  for (size_t k = 0; k < (size_t)H0 * H1; ++k) grad[pF1 + k] = acc[t->o_W1f + k];
  for (int k = 0; k < H1; ++k) grad[pfb1 + k] = acc[t->o_b1f + k];
  for (int k = 0; k < H1; ++k) grad[pwo + k] = acc[t->o_wout + k];
  std::vector<int> cnt(T, 0);
  for (int k = 0; k < N; ++k) cnt[types[k]] += 1;
  for (int f = 0; f < B; ++f) {
    grad[pbo] += (double)av[f] * N;
    for (int a = 0; a < T; ++a) grad[peb + a] += (double)av[f] * cnt[a];
  }
  return DP_OK;
}

int check_batch(const dp_trainer *t, const double *d_frames, const int32_t *d_types, int natoms,
                int nframes, const double *d_e_label, const double *d_f_label, const double *loss) {
  if (!t) return fail(DP_ERR_ARG, "trainer handle is NULL");
  if (natoms < 1 || nframes < 1) return fail(DP_ERR_ARG, "natoms and nframes must be >= 1");
  if ((long)natoms * t->m->sel > (1L << 28)) return fail(DP_ERR_ARG, "natoms * sel too large");
  if (!d_frames || !d_types || !d_e_label || !d_f_label || !loss)
    return fail(DP_ERR_ARG, "an array pointer is NULL");
  return DP_OK;
}

}  // namespace

extern "C" {

int dp_train_create(const char *weights_path, double rcut, int sel, const dp_train_options *opt,
                    dp_trainer **out) {
  if (!out || !opt) return fail(DP_ERR_ARG, "out/opt is NULL");
  *out = nullptr;
  if (!(opt->pref_e >= 0) || !(opt->pref_f >= 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) ||
      !(opt->beta2 >= 0 && opt->beta2 < 1) || !(opt->eps > 0))
    return fail(DP_ERR_ARG, "bad training options");
  if (opt->precision != DP_PREC_FP32 && opt->precision != DP_PREC_BF16)
    return fail(DP_ERR_ARG, "unknown precision %d", opt->precision);
  dp_model *m = nullptr;
  int rc = dp_create(weights_path, rcut, sel, &m);
  if (rc) return rc;
  dp_trainer *t = new dp_trainer();
  t->m = m;
  t->opt = *opt;
  auto bail = [&](int code) {
    delete t;
    return code;
  };
  const bool fit_ok = m->fit.size() == 2 && m->fit[0] == m->fit[1] &&
                      (m->fit[0] == 32 || m->fit[0] == 64 || m->fit[0] == 128 ||
                       m->fit[0] == 256);
  if (m->n_attn != 0 || m->emb.size() != 3 || m->emb[0] != kTrN1 || m->emb[1] != kTrN2 ||
      m->emb[2] != kTrN3 || !fit_ok || m->ntypes * m->ntypes > 64)
    return bail(fail(DP_ERR_WEIGHTS,
                     "the trainer takes an attention-free model with embedding 16/32/64, two "
                     "equal fitting layers of width 32, 64, 128 or 256 and at most 8 types"));
  if ((rc = dp_set_precision(m, opt->precision))) return bail(rc);
  tensor_list(m, t);
  // header and FP32 masters from the file
  {
    FILE *f = fopen(weights_path, "rb");
    if (!f) return bail(fail(DP_ERR_WEIGHTS, "cannot reopen '%s'", weights_path));
    std::vector<char> buf;
    char tmp[1 << 16];
    size_t n;
    while ((n = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + n);
    fclose(f);
    const size_t body = sizeof(double) * (size_t)t->nparams;
    if (buf.size() < body + 8) return bail(fail(DP_ERR_WEIGHTS, "weights file too short"));
    const size_t h = buf.size() - body;
    t->header.assign(buf.begin(), buf.begin() + h);
    t->theta_h.resize(t->nparams);
    for (int k = 0; k < t->nparams; ++k) {
      double v;
      memcpy(&v, buf.data() + h + sizeof(double) * k, sizeof(double));
      t->theta_h[k] = (float)v;
    }
  }
  // the inference weights are rebuilt from the FP32 masters (their values as FP64)
  if ((rc = load_weights_image(m, make_image(t), true))) return bail(rc);
  const size_t np = (size_t)t->nparams;
  const int T = m->ntypes, H = m->fit[0], nd = m->M * m->axis;
  size_t o = 0;
  auto slot = [&](size_t n) {
    const size_t r = o;
    o += n;
    return r;
  };
  t->o_W2 = slot((size_t)kTrN1 * kTrN2);
  t->o_b2 = slot(kTrN2);
  t->o_W3 = slot((size_t)kTrN2 * kTrN3);
  t->o_b3 = slot(kTrN3);
  t->o_tab = slot((size_t)T * T * kTrN1);
  t->o_ws = slot(kTrN1);
  t->o_W0d = slot((size_t)nd * H);
  t->o_fb0 = slot((size_t)T * H);
  t->o_W1f = slot((size_t)H * H);
  t->o_b1f = slot(H);
  t->o_wout = slot(H);
  t->acc_n = o;
  hipError_t e = hipMalloc(&t->theta, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&t->am, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&t->av, sizeof(float) * np);
  if (e == hipSuccess) e = hipMalloc(&t->grad_d, sizeof(double) * np);
  if (e == hipSuccess) e = hipMalloc(&t->acc, sizeof(double) * t->acc_n);
  if (e == hipSuccess) e = hipMemcpy(t->theta, t->theta_h.data(), sizeof(float) * np,
                                     hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(t->am, 0, sizeof(float) * np);
  if (e == hipSuccess) e = hipMemset(t->av, 0, sizeof(float) * np);
  if (e != hipSuccess)
    return bail(fail(e == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_DEVICE,
                     "trainer setup failed: %s", hipGetErrorString(e)));
  *out = t;
  return DP_OK;
}

int dp_train_gradient(dp_trainer *t, const double *d_frames, const int32_t *d_types,
                      const double *box, int natoms, int nframes, const double *d_e_label,
                      const double *d_f_label, double *loss, double *grad, void *hip_stream) {
  int rc = check_batch(t, d_frames, d_types, natoms, nframes, d_e_label, d_f_label, loss);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(t->m->device));
  std::vector<double> g;
  if ((rc = batch_gradient(t, d_frames, d_types, box, natoms, nframes, d_e_label, d_f_label, loss,
                           g, (hipStream_t)hip_stream)))
    return rc;
  if (grad) memcpy(grad, g.data(), sizeof(double) * g.size());
  return DP_OK;
}

int dp_train_step(dp_trainer *t, const double *d_frames, const int32_t *d_types,
                  const double *box, int natoms, int nframes, const double *d_e_label,
                  const double *d_f_label, double lr, double *loss, void *hip_stream) {
  int rc = check_batch(t, d_frames, d_types, natoms, nframes, d_e_label, d_f_label, loss);
  if (rc) return rc;
  if (!(lr >= 0) || !std::isfinite(lr)) return fail(DP_ERR_ARG, "bad learning rate");
  HIP_TRY(hipSetDevice(t->m->device));
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<double> g;
  if ((rc = batch_gradient(t, d_frames, d_types, box, natoms, nframes, d_e_label, d_f_label, loss,
                           g, s)))
    return rc;
  const int np = t->nparams;
  HIP_TRY(hipMemcpyAsync(t->grad_d, g.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
  t->adam_t += 1;
  const double b1 = t->opt.beta1, b2 = t->opt.beta2;
  const float bc1 = (float)(1.0 - std::pow(b1, t->adam_t));
  const float bc2 = (float)(1.0 - std::pow(b2, t->adam_t));
  launch_adam(t->theta, t->am, t->av, t->grad_d, np, (float)lr, (float)b1, (float)b2,
              (float)t->opt.eps, bc1, bc2, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(t->theta_h.data(), t->theta, sizeof(float) * np, hipMemcpyDeviceToHost,
                         s));
  HIP_TRY(hipStreamSynchronize(s));
  return load_weights_image(t->m, make_image(t), true);
}

int dp_train_params(const dp_trainer *t, double *params, int32_t *nparams) {
  if (!t || !nparams) return fail(DP_ERR_ARG, "NULL argument");
  *nparams = t->nparams;
  if (params)
    for (int k = 0; k < t->nparams; ++k) params[k] = (double)t->theta_h[k];
  return DP_OK;
}

int dp_train_save(const dp_trainer *t, const char *path) {
  if (!t || !path) return fail(DP_ERR_ARG, "NULL argument");
  const std::vector<char> img = make_image(t);
  FILE *f = fopen(path, "wb");
  if (!f) return fail(DP_ERR_WEIGHTS, "cannot write '%s'", path);
  const size_t n = fwrite(img.data(), 1, img.size(), f);
  const int cl = fclose(f);
  if (n != img.size() || cl != 0) return fail(DP_ERR_WEIGHTS, "short write to '%s'", path);
  return DP_OK;
}

int dp_train_checkpoint(const dp_trainer *t, const char *path) {
  if (!t || !path) return fail(DP_ERR_ARG, "NULL argument");
  HIP_TRY(hipSetDevice(t->m->device));
  const size_t np = (size_t)t->nparams;
  std::vector<float> mv(2 * np);
  HIP_TRY(hipMemcpy(mv.data(), t->am, sizeof(float) * np, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(mv.data() + np, t->av, sizeof(float) * np, hipMemcpyDeviceToHost));
  FILE *f = fopen(path, "wb");
  if (!f) return fail(DP_ERR_WEIGHTS, "cannot write '%s'", path);
  const int32_t head[2] = {t->nparams, t->adam_t};
  bool ok = fwrite("DPA1TRN\0", 1, 8, f) == 8 && fwrite(head, sizeof(head), 1, f) == 1 &&
            fwrite(t->theta_h.data(), sizeof(float), np, f) == np &&
            fwrite(mv.data(), sizeof(float), 2 * np, f) == 2 * np;
  ok = (fclose(f) == 0) && ok;
  return ok ? DP_OK : fail(DP_ERR_WEIGHTS, "short write to '%s'", path);
}

int dp_train_resume(dp_trainer *t, const char *path) {
  if (!t || !path) return fail(DP_ERR_ARG, "NULL argument");
  FILE *f = fopen(path, "rb");
  if (!f) return fail(DP_ERR_WEIGHTS, "cannot open '%s'", path);
  char magic[8] = {0};
  int32_t head[2] = {0, 0};
  const size_t np = (size_t)t->nparams;
  std::vector<float> th(np), mv(2 * np);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "DPA1TRN\0", 8) == 0 &&
            fread(head, sizeof(head), 1, f) == 1 && head[0] == t->nparams && head[1] >= 0 &&
            fread(th.data(), sizeof(float), np, f) == np &&
            fread(mv.data(), sizeof(float), 2 * np, f) == 2 * np;
  char extra;
  ok = ok && fread(&extra, 1, 1, f) == 0;
  fclose(f);
  if (!ok) return fail(DP_ERR_WEIGHTS, "'%s' is not a checkpoint of this trainer", path);
  HIP_TRY(hipSetDevice(t->m->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(t->theta, th.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t->am, mv.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(t->av, mv.data() + np, sizeof(float) * np, hipMemcpyHostToDevice));
  t->theta_h = th;
  t->adam_t = head[1];
  return load_weights_image(t->m, make_image(t), true);
}

void dp_train_destroy(dp_trainer *t) {
  if (!t) return;
  (void)hipSetDevice(t->m->device);
  (void)hipDeviceSynchronize();
  delete t;
}

int dp_force_error(const double *d_a, const double *d_b, int n, double *rmse_max,
                   void *hip_stream) {
  if (!rmse_max || n < 0 || (n > 0 && (!d_a || !d_b)))
    return fail(DP_ERR_ARG, "bad arguments");
  if (n > DP_FORCE_ERROR_MAX_ATOMS)
    return fail(DP_ERR_ARG, "n = %d exceeds DP_FORCE_ERROR_MAX_ATOMS (%d)", n,
                DP_FORCE_ERROR_MAX_ATOMS);
  rmse_max[0] = rmse_max[1] = 0.0;
  if (n == 0) return DP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  const int nb = force_error_blocks(n);
  double *part = nullptr;
  HIP_TRY(hipMalloc(&part, sizeof(double) * 2 * nb));
  launch_force_error(d_a, d_b, n, part, s);
  std::vector<double> h(2 * nb);
  hipError_t e = hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part);
  if (e != hipSuccess) return fail(DP_ERR_DEVICE, "force error: %s", hipGetErrorString(e));
  double sq = 0.0, mx = 0.0;
  for (int b = 0; b < nb; ++b) {
    sq += h[2 * b];
    mx = std::max(mx, h[2 * b + 1]);
  }
  rmse_max[0] = std::sqrt(sq / (3.0 * n));
  rmse_max[1] = mx;
  return DP_OK;
}

}  // extern "C"
