// Host side of the DPA-1 library: weights, workspace, launch sequence and
// the C ABI declared in include/dpa1.h.
//
// One step (Sec. II-B model; Sec. II-C local/ghost semantics):
//   cell binning -> full neighbour lists -> per-pair geometry and first
//   embedding layer -> embedding layers -> [QKV projection -> attention core
//   -> output projection + layer norm + residual] x n_attn -> descriptor ->
//   fitting net -> atomic energies; then the input-gradient adjoint in
//   reverse order down to g_ij = de_i/dd_ij, and forces/virial by gather.
// Everything is enqueued on one stream; the step allocates nothing once the
// workspace has grown to the system size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dpa1.h"
#include "dpa1_internal.h"
#include "dpa1_model.h"

using namespace dpa1;

namespace {
thread_local std::string g_err;
}  // namespace

int dpa1::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace {

// --------------------------------------------------------------------- weights

struct Reader {
  const std::vector<char> &buf;
  size_t off = 0;
  bool ok = true;
  template <class T>
  T get() {
    T v{};
    if (off + sizeof(T) > buf.size()) {
      ok = false;
      return v;
    }
    memcpy(&v, buf.data() + off, sizeof(T));
    off += sizeof(T);
    return v;
  }
  std::vector<double> arr(size_t n) {
    std::vector<double> v(n);
    if (off + 8 * n > buf.size()) {
      ok = false;
      return v;
    }
    memcpy(v.data(), buf.data() + off, 8 * n);
    off += 8 * n;
    return v;
  }
};

// Uploads h to a new device array, or overwrites *out in place when it is set
// (a weights refresh keeps every array and its size).
int upload(dp_model *m, const std::vector<float> &h, float **out) {
  void *p = *out;
  if (!p) {
    HIP_TRY(hipMalloc(&p, std::max<size_t>(h.size(), 1) * sizeof(float)));
    m->weight_allocs.push_back(p);
  }
  HIP_TRY(hipMemcpy(p, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  *out = (float *)p;
  return DP_OK;
}

// W is [fin][fout] row-major FP64.
int make_linear(dp_model *m, const std::vector<double> &W, const std::vector<double> &b, int fin,
                int fout, int ldin, int ldout, Linear &L) {
  L.fin = fin;
  L.fout = fout;
  L.ldin = ldin;
  L.ldout = ldout;
  L.res = residual_rule(fin, fout);
  std::vector<float> wt((size_t)ldout * ldin, 0.f), wb((size_t)ldin * ldout, 0.f),
      bb(ldout, 0.f);
  for (int k = 0; k < fin; ++k)
    for (int o = 0; o < fout; ++o) {
      const float v = (float)W[(size_t)k * fout + o];
      wt[(size_t)o * ldin + k] = v;
      wb[(size_t)k * ldout + o] = v;
    }
  for (int o = 0; o < fout; ++o) bb[o] = (float)b[o];
  int rc;
  if ((rc = upload(m, wt, &L.Wt))) return rc;
  if ((rc = upload(m, wb, &L.Wb))) return rc;
  return upload(m, bb, &L.b);
}

}  // namespace

int dpa1::load_weights_image(dp_model *m, const std::vector<char> &buf, bool refresh) {
  if (buf.size() < 8 || memcmp(buf.data(), "DPA1WTS\0", 8) != 0)
    return fail(DP_ERR_WEIGHTS, "not a DPA-1 weights image");
  Reader rd{buf, 8};
  const uint32_t version = rd.get<uint32_t>();
  const uint32_t n_int = rd.get<uint32_t>();
  if (!rd.ok || version != 1) return fail(DP_ERR_WEIGHTS, "unsupported weights version");
  if (n_int < 7 || n_int > 64) return fail(DP_ERR_WEIGHTS, "bad header size");
  std::vector<int> ints(n_int);
  for (auto &v : ints) v = rd.get<int32_t>();
  const uint32_t n_dbl = rd.get<uint32_t>();
  if (!rd.ok || n_dbl < 3 || n_dbl > 64) return fail(DP_ERR_WEIGHTS, "bad header");
  std::vector<double> dbls(n_dbl);
  for (auto &v : dbls) v = rd.get<double>();
  if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated header");
  if (refresh) {
    std::vector<int> cur = {m->ntypes, m->tebd, m->axis, m->n_attn, m->dattn,
                            (int)m->emb.size(), (int)m->fit.size()};
    cur.insert(cur.end(), m->emb.begin(), m->emb.end());
    cur.insert(cur.end(), m->fit.begin(), m->fit.end());
    if (cur != ints) return fail(DP_ERR_WEIGHTS, "weights image shape differs from the model");
  }
  m->ntypes = ints[0];
  m->tebd = ints[1];
  m->axis = ints[2];
  m->n_attn = ints[3];
  m->dattn = ints[4];
  const int n_emb = ints[5], n_fit = ints[6];
  if (n_emb < 2 || n_fit < 1 || (size_t)(7 + n_emb + n_fit) != n_int)
    return fail(DP_ERR_WEIGHTS, "unsupported layer counts (embedding %d, fitting %d)", n_emb,
                n_fit);
  m->emb.assign(ints.begin() + 7, ints.begin() + 7 + n_emb);
  m->fit.assign(ints.begin() + 7 + n_emb, ints.end());
  m->rcut_smth = dbls[0];
  m->shift = dbls[1];
  m->ln_eps = dbls[2];
  m->M = m->emb.back();
  if (m->ntypes < 1 || m->ntypes > 128 || m->tebd < 1 || m->tebd > 256)
    return fail(DP_ERR_WEIGHTS, "bad type embedding shape");
  for (int w : m->emb)
    if (w < 1 || w > 128) return fail(DP_ERR_WEIGHTS, "embedding widths must be in [1, 128]");
  for (int w : m->fit)
    if (w < 1 || w > 4096) return fail(DP_ERR_WEIGHTS, "bad fitting width");
  if (m->axis < 1 || m->axis > m->M || m->axis > 16)
    return fail(DP_ERR_WEIGHTS, "axis width must be in [1, min(16, M)]");
  if (m->n_attn < 0 || m->n_attn > 16) return fail(DP_ERR_WEIGHTS, "bad attention layer count");
  if (m->n_attn > 0 && m->dattn != 128)
    return fail(DP_ERR_WEIGHTS, "attention width %d unsupported (the attention kernels take 128)", m->dattn);
  const int x0 = 1 + 2 * m->tebd;
  if (residual_rule(x0, m->emb[0]) != RES_NONE)
    return fail(DP_ERR_WEIGHTS, "a residual on the first embedding layer is unsupported");
  const int fin0 = m->M * m->axis + m->tebd;
  if (residual_rule(fin0, m->fit[0]) != RES_NONE)
    return fail(DP_ERR_WEIGHTS, "a residual on the first fitting layer is unsupported");
  if (n_fit >= 2 && residual_rule(m->fit[n_fit - 2], m->fit[n_fit - 1]) == RES_DOUBLE)
    return fail(DP_ERR_WEIGHTS, "a doubling residual on the last fitting layer is unsupported");
  if (!(m->ln_eps >= 0) || !std::isfinite(m->shift) || !(m->rcut_smth >= 0))
    return fail(DP_ERR_WEIGHTS, "bad scalar parameters");

  m->lde.clear();
  m->ldf.clear();
  for (int w : m->emb) m->lde.push_back(pad16(w));
  for (int w : m->fit) m->ldf.push_back(pad16(w));
  m->ldM = pad16(m->M);
  m->ldD = pad16(m->M * m->axis);
  const int T = m->ntypes, E = m->tebd;
  int rc;
  // type embedding and the first embedding layer folded into a table
  auto temb = rd.arr((size_t)T * E);
  auto W1 = rd.arr((size_t)x0 * m->emb[0]);
  auto b1 = rd.arr(m->emb[0]);
  if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated weights");
  {
    const int n1 = m->emb[0], ld = m->lde[0];
    std::vector<float> table((size_t)T * T * ld, 0.f), wsv(ld, 0.f);
    for (int a = 0; a < T; ++a)      // neighbour type
      for (int b = 0; b < T; ++b)    // centre type
        for (int o = 0; o < n1; ++o) {
          double v = b1[o];
          for (int k = 0; k < E; ++k) {
            v += temb[(size_t)a * E + k] * W1[(size_t)(1 + k) * n1 + o];
            v += temb[(size_t)b * E + k] * W1[(size_t)(1 + E + k) * n1 + o];
          }
          table[((size_t)a * T + b) * ld + o] = (float)v;
        }
    for (int o = 0; o < n1; ++o) wsv[o] = (float)W1[o];
    if ((rc = upload(m, table, &m->type_table))) return rc;
    if ((rc = upload(m, wsv, &m->ws))) return rc;
  }
  m->embl.resize(n_emb);
  for (int l = 1; l < n_emb; ++l) {
    auto W = rd.arr((size_t)m->emb[l - 1] * m->emb[l]);
    auto b = rd.arr(m->emb[l]);
    if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated weights");
    if ((rc = make_linear(m, W, b, m->emb[l - 1], m->emb[l], m->lde[l - 1], m->lde[l],
                          m->embl[l])))
      return rc;
  }
  const int Mw = m->M, D = m->dattn, ldM = m->ldM;
  for (int a = 0; a < m->n_attn; ++a) {
    std::vector<double> Wq = rd.arr((size_t)Mw * D), bq = rd.arr(D);
    std::vector<double> Wk = rd.arr((size_t)Mw * D), bk = rd.arr(D);
    std::vector<double> Wv = rd.arr((size_t)Mw * D), bv = rd.arr(D);
    std::vector<double> Wo = rd.arr((size_t)D * Mw), bo = rd.arr(Mw);
    std::vector<double> ga = rd.arr(Mw), be = rd.arr(Mw);
    if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated weights");
    dp_model::Attn at = refresh ? m->attn[a] : dp_model::Attn{};
    std::vector<float> wt((size_t)3 * D * ldM, 0.f), wb((size_t)ldM * 3 * D, 0.f),
        bqkv(3 * D, 0.f);
    const std::vector<double> *Ws[3] = {&Wq, &Wk, &Wv};
    const std::vector<double> *Bs[3] = {&bq, &bk, &bv};
    for (int s = 0; s < 3; ++s) {
      for (int k = 0; k < Mw; ++k)
        for (int o = 0; o < D; ++o) {
          const float v = (float)(*Ws[s])[(size_t)k * D + o];
          wt[(size_t)(s * D + o) * ldM + k] = v;
          wb[(size_t)k * 3 * D + s * D + o] = v;
        }
      for (int o = 0; o < D; ++o) bqkv[s * D + o] = (float)(*Bs[s])[o];
    }
    std::vector<float> wto((size_t)ldM * D, 0.f), wbo((size_t)D * ldM, 0.f), bov(ldM, 0.f),
        gav(ldM, 0.f), bev(ldM, 0.f);
    for (int k = 0; k < D; ++k)
      for (int o = 0; o < Mw; ++o) {
        const float v = (float)Wo[(size_t)k * Mw + o];
        wto[(size_t)o * D + k] = v;
        wbo[(size_t)k * ldM + o] = v;
      }
    for (int o = 0; o < Mw; ++o) {
      bov[o] = (float)bo[o];
      gav[o] = (float)ga[o];
      bev[o] = (float)be[o];
    }
    if ((rc = upload(m, wt, &at.Wt_qkv)) || (rc = upload(m, wb, &at.Wb_qkv)) ||
        (rc = upload(m, bqkv, &at.b_qkv)) || (rc = upload(m, wto, &at.Wt_o)) ||
        (rc = upload(m, wbo, &at.Wb_o)) || (rc = upload(m, bov, &at.b_o)) ||
        (rc = upload(m, gav, &at.gamma)) || (rc = upload(m, bev, &at.beta)))
      return rc;
    if (refresh)
      m->attn[a] = at;
    else
      m->attn.push_back(at);
  }
  m->fitl.resize(n_fit);
  {
    const int nd = Mw * m->axis;
    auto W = rd.arr((size_t)fin0 * m->fit[0]);
    auto b = rd.arr(m->fit[0]);
    if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated weights");
    std::vector<double> Wd(W.begin(), W.begin() + (size_t)nd * m->fit[0]);
    if ((rc = make_linear(m, Wd, b, nd, m->fit[0], m->ldD, m->ldf[0], m->fitl[0]))) return rc;
    m->fitl[0].res = RES_NONE;
    std::vector<float> fb((size_t)T * m->ldf[0], 0.f);
    for (int a = 0; a < T; ++a)
      for (int o = 0; o < m->fit[0]; ++o) {
        double v = b[o];
        for (int k = 0; k < E; ++k)
          v += temb[(size_t)a * E + k] * W[(size_t)(nd + k) * m->fit[0] + o];
        fb[(size_t)a * m->ldf[0] + o] = (float)v;
      }
    if ((rc = upload(m, fb, &m->fb0))) return rc;
  }
  for (int l = 1; l < n_fit; ++l) {
    auto W = rd.arr((size_t)m->fit[l - 1] * m->fit[l]);
    auto b = rd.arr(m->fit[l]);
    if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated weights");
    if ((rc = make_linear(m, W, b, m->fit[l - 1], m->fit[l], m->ldf[l - 1], m->ldf[l],
                          m->fitl[l])))
      return rc;
  }
  {
    auto wo = rd.arr(m->fit.back());
    auto bo = rd.arr(1);
    auto eb = rd.arr(T);
    if (!rd.ok) return fail(DP_ERR_WEIGHTS, "truncated weights");
    if (rd.off != buf.size()) return fail(DP_ERR_WEIGHTS, "weights file has trailing bytes");
    std::vector<float> wov(m->ldf.back(), 0.f), ebv(T);
    for (int o = 0; o < m->fit.back(); ++o) wov[o] = (float)wo[o];
    for (int a = 0; a < T; ++a) ebv[a] = (float)eb[a];
    m->b_out = (float)bo[0];
    if ((rc = upload(m, wov, &m->w_out))) return rc;
    if ((rc = upload(m, ebv, &m->ebias))) return rc;
  }
  return DP_OK;
}

namespace {

int load_weights(dp_model *m, const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) return fail(DP_ERR_WEIGHTS, "cannot open weights file '%s'", path);
  std::vector<char> buf;
  char tmp[1 << 16];
  size_t n;
  while ((n = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + n);
  fclose(f);
  if (buf.size() < 8 || memcmp(buf.data(), "DPA1WTS\0", 8) != 0)
    return fail(DP_ERR_WEIGHTS, "'%s' is not a DPA-1 weights file", path);
  return load_weights_image(m, buf, false);
}

// ------------------------------------------------------------------- workspace

struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

// The workspace is two arenas.  The topology arena holds the per-atom and
// per-centre buffers (coordinates, cell lists, neighbour lists, descriptor,
// fitting net), laid out for nloc / nall / ncell.  The pair arena holds every
// per-pair buffer (geometry, embedding, attention and their adjoints) for a
// capacity of P pair rows, taken from the real neighbour-pair count of the
// step that lays it out plus 1/8 headroom (and never more than nloc * sel),
// instead of nloc * sel rows.  With base == nullptr the carvers only measure.
// With shared set, every attention layer uses one set of QKV, attention-
// output, logit and softmax-statistics buffers (the adjoint recomputes them).
// The fused embedding kernels keep no hidden-layer activations, so their
// per-layer buffers are not laid out.
bool emb_is_fused(const dp_model *m) {
  return m->emb.size() == 3 && emb_fused_supported(m->lde[0], m->lde[1], m->lde[2]);
}

size_t carve_topo(dp_model *m, char *base, int nloc, int nall, int ncell) {
  Carver c{base};
  auto &w = m->w;
  const size_t NL = (size_t)nloc + 16;
  w.coords = c.take<double>(3 * (size_t)nall);
  w.types = c.take<int32_t>(nall);
  w.types_safe = c.take<int32_t>(nall);
  w.out_e = c.take<double>(1);
  w.out_f = c.take<double>(3 * (size_t)nall);
  w.out_v = c.take<double>(9);
  w.out_ae = c.take<double>(nloc);
  w.vir_part = c.take<double>(9 * (size_t)nloc);
  w.atom_cell = c.take<int>(nall);
  w.cell_count = c.take<int>(ncell);
  w.cell_start = c.take<int>(ncell + 1);
  w.cell_fill = c.take<int>(ncell);
  w.cell_atoms = c.take<int>(nall);
  w.nlist = c.take<int>((size_t)nall * m->sel);
  w.nnei = c.take<int>(nall);
  w.pair_off = c.take<int>(nloc + 1);
  w.ccount = c.take<int>(8);
  w.clist = c.take<int>(4 * (size_t)nloc);
  w.T = c.take<float>(NL * 4 * m->M);
  w.dmat = c.take<float>(NL * m->ldD);
  w.e = c.take<float>(NL);
  const int nf = (int)m->fit.size();
  w.z.assign(nf, nullptr);
  w.tf.assign(nf, nullptr);
  w.fa.assign(nf, nullptr);
  w.fdz.assign(nf, nullptr);
  for (int l = 0; l < nf; ++l) {
    w.z[l] = c.take<float>(NL * m->ldf[l]);
    w.tf[l] = c.take<float>(NL * m->ldf[l]);
    w.fa[l] = c.take<float>(NL * m->ldf[l]);
    w.fdz[l] = c.take<float>(NL * m->ldf[l]);
  }
  w.dD = c.take<float>(NL * m->ldD);
  return c.off + 256;
}

size_t carve_pairs(dp_model *m, char *base, size_t P, bool shared) {
  Carver c{base};
  auto &w = m->w;
  const bool fused = emb_is_fused(m);
  w.geom = c.take<float>(P * kGeom);
  const int ne = (int)m->emb.size();
  w.h.assign(ne, nullptr);
  w.te.assign(ne, nullptr);
  for (int l = 0; l < ne; ++l) {
    // fused: only the first layer's output (the adjoint's recomputation
    // input) and the last one (G) are stored
    if (fused && l > 0 && l < ne - 1) continue;
    w.h[l] = c.take<float>(P * m->lde[l]);
    w.te[l] = l == 0 ? w.h[0] : (fused ? nullptr : c.take<float>(P * m->lde[l]));
  }
  const int na = m->n_attn;
  w.qkv.assign(na, nullptr);
  w.o.assign(na, nullptr);
  w.lam.assign(na, nullptr);
  w.fstat.assign(na, nullptr);
  w.xhat.assign(na, nullptr);
  w.rstd.assign(na, nullptr);
  w.G.assign(na + 1, nullptr);
  w.G[0] = w.h[ne - 1];
  for (int a = 0; a < na; ++a) {
    if (shared && a > 0) {
      w.qkv[a] = w.qkv[0];
      w.o[a] = w.o[0];
      w.lam[a] = w.lam[0];
      w.fstat[a] = w.fstat[0];
    } else {
      w.qkv[a] = c.take<float>(P * 3 * m->dattn);
      w.o[a] = c.take<float>(P * m->dattn);
      w.lam[a] = c.take<float>(P * kAttnLamLd);
      w.fstat[a] = c.take<float>(P * 2);
    }
    w.xhat[a] = c.take<float>(P * m->ldM);
    w.rstd[a] = c.take<float>(P);
    w.G[a + 1] = c.take<float>(P * m->ldM);
  }
  w.dGa = c.take<float>(P * m->ldM);
  w.dGb = c.take<float>(P * m->ldM);
  w.dY = c.take<float>(P * m->ldM);
  w.dO = c.take<float>(P * std::max(m->dattn, 16));
  w.dqkv = c.take<float>(P * 3 * std::max(m->dattn, 16));
  w.dRt = c.take<float>(P * 4);
  w.gw = c.take<float>(P);
  w.gr = c.take<float>(P * 4);
  w.gs = c.take<float>(P);
  w.g = c.take<float>(P * 4);
  w.astat = c.take<float>(P * 4);
  w.qside = c.take<float>(P * 4);
  w.dA = m->n_attn > 0 ? c.take<float>(P * kAttnLamLd) : nullptr;
  w.du.assign(ne, nullptr);
  w.dh.assign(ne, nullptr);
  if (!fused)
    for (int l = 0; l < ne; ++l) {
      w.du[l] = c.take<float>(P * m->lde[l]);
      w.dh[l] = c.take<float>(P * m->lde[l]);
    }
  return c.off + 256;
}

int free_arenas(dp_model *m) {
  if (m->arena || m->parena) HIP_TRY(hipDeviceSynchronize());
  if (m->arena) HIP_TRY(hipFree(m->arena));
  if (m->parena) HIP_TRY(hipFree(m->parena));
  m->arena = m->parena = nullptr;
  m->arena_bytes = m->parena_bytes = 0;
  m->cap_nloc = m->cap_nall = m->cap_ncell = -1;
  m->cap_pairs = -1;
  m->fwd.valid = false;
  return DP_OK;
}

int ensure_workspace(dp_model *m, int nloc, int nall, int ncell) {
  // the topology layout is fixed for the capacity until it grows or the
  // budget changes; the pair arena is laid out by the forward, from the
  // step's real pair count
  if (m->arena && nloc <= m->cap_nloc && nall <= m->cap_nall && ncell <= m->cap_ncell)
    return DP_OK;
  const int cl = std::max(nloc, m->cap_nloc), ca = std::max(nall, m->cap_nall),
            cc = std::max(ncell, m->cap_ncell);
  int rc;
  if ((rc = free_arenas(m))) return rc;
  const size_t bytes = carve_topo(m, nullptr, cl, ca, cc);
  if (m->mem_budget > 0 && (double)bytes > m->mem_budget)
    return fail(DP_ERR_OOM, "workspace of %zu bytes exceeds the memory budget of %.0f bytes",
                bytes, m->mem_budget);
  HIP_TRY(hipMalloc(&m->arena, bytes));
  HIP_TRY(hipMemset(m->arena, 0, bytes));
  m->arena_bytes = bytes;
  carve_topo(m, (char *)m->arena, cl, ca, cc);
  m->cap_nloc = cl;
  m->cap_nall = ca;
  m->cap_ncell = cc;
  return DP_OK;
}

// Lays out the pair arena for at least `pairs` rows (synchronous; the caller
// has synchronised the stream).  Every layer's attention activations are
// stored unless that exceeds the memory budget (then shared buffers and
// recomputation in the adjoint).
int ensure_pairs(dp_model *m, long pairs) {
  const long cap_max = (long)m->cap_nloc * m->sel;
  long cap = pairs + pairs / 8;
  cap = std::min(std::max(cap, pairs), cap_max);
  const size_t P = (size_t)cap + 64;
  const dp_model::WS saved = m->w;
  const size_t full = carve_pairs(m, nullptr, P, false);
  const bool shared = m->n_attn > 1 && m->mem_budget > 0 &&
                      (double)(full + m->arena_bytes) > m->mem_budget;
  const size_t bytes = shared ? carve_pairs(m, nullptr, P, true) : full;
  m->w = saved;
  if (m->mem_budget > 0 && (double)(bytes + m->arena_bytes) > m->mem_budget)
    return fail(DP_ERR_OOM, "workspace of %zu bytes exceeds the memory budget of %.0f bytes%s",
                bytes + m->arena_bytes, m->mem_budget,
                m->n_attn > 1 ? " even with recomputation" : "");
  if (m->parena) {
    HIP_TRY(hipFree(m->parena));
    m->parena = nullptr;
    m->parena_bytes = 0;
  }
  HIP_TRY(hipMalloc(&m->parena, bytes));
  HIP_TRY(hipMemset(m->parena, 0, bytes));
  m->parena_bytes = bytes;
  carve_pairs(m, (char *)m->parena, P, shared);
  m->recompute = shared;
  m->cap_pairs = cap;
  m->cap_pairs_nloc = m->cap_nloc;
  m->want_pairs = 0;
  m->fwd.valid = false;
  return DP_OK;
}

// ---------------------------------------------------------------- validation

int make_grid(const dp_model *m, const double *box, const double *bbox_lo,
              const double *bbox_hi, CellGrid &g) {
  memset(&g, 0, sizeof(g));
  const double edge_min = m->rcut * (1.0 + 1e-9);
  if (box) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        if (!std::isfinite(box[3 * a + b])) return fail(DP_ERR_BOX, "box is not finite");
        if (a != b && box[3 * a + b] != 0.0)
          return fail(DP_ERR_BOX, "only orthorhombic boxes are supported");
      }
    g.periodic = 1;
    for (int a = 0; a < 3; ++a) {
      const double L = box[4 * a];
      if (!(L > 2.0 * m->rcut))
        return fail(DP_ERR_BOX, "box length %g must exceed 2*rcut = %g", L, 2.0 * m->rcut);
      int nc = (int)std::floor(L / edge_min);
      nc = std::max(1, std::min(nc, 1024));
      g.nc[a] = nc;
      g.L[a] = L;
      g.lo[a] = 0.0;
      g.inv_edge[a] = nc / L;
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      const double ext = bbox_hi[a] - bbox_lo[a];
      int nc = ext > 0 ? (int)std::floor(ext / edge_min) : 1;
      nc = std::max(1, std::min(nc, 128));
      g.nc[a] = nc;
      g.lo[a] = bbox_lo[a];
      g.L[a] = 0.0;
      g.inv_edge[a] = ext > 0 ? nc / ext : 0.0;
    }
  }
  g.ncell = g.nc[0] * g.nc[1] * g.nc[2];
  return DP_OK;
}

__global__ void k_fill_int(int *p, int n, int v) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}
// Start of a step: the flags and attention class counts (block 0) and the
// per-cell atom counters of the binning (all blocks), in one launch.
__global__ void k_init_step(DevFlags *f, int *ccount, int *cell_count, int *cell_fill,
                            int ncell) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      f->overflow_atom = INT_MAX;
      f->overflow_count = 0;
      f->bad_type_atom = INT_MAX;
      f->pair_overflow = 0;
    }
    if (threadIdx.x < 8) ccount[threadIdx.x] = 0;
  }
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ncell) {
    cell_count[k] = 0;
    cell_fill[k] = 0;
  }
}
// Capacity check of the pair arena (one block): a step with more neighbour
// pairs than the arena holds records its count and gets no pair work at all
// (every neighbour count, locals and ghosts, and every pair offset set to 0),
// so no kernel indexes past the arena; the workspace grows at the next call.
__global__ __launch_bounds__(1024) void k_pair_guard(int *pair_off, int *nnei, int nloc, int nall,
                                                     long cap, DevFlags *f) {
  const int total = pair_off[nloc];
  __syncthreads();  // every thread has read the total before any is cleared
  if ((long)total <= cap) return;
  if (threadIdx.x == 0) f->pair_overflow = total;
  for (int k = threadIdx.x; k < nall; k += blockDim.x) nnei[k] = 0;
  for (int k = threadIdx.x; k <= nloc; k += blockDim.x) pair_off[k] = 0;
}
__global__ void k_bbox(const double *x, int n, double *out) {
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = t; k < n; k += 256)
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], x[3 * k + c]);
      hi[c] = fmax(hi[c], x[3 * k + c]);
    }
  for (int c = 0; c < 3; ++c) {
    red[c][t] = lo[c];
    red[3 + c][t] = hi[c];
  }
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h)
      for (int c = 0; c < 3; ++c) {
        red[c][t] = fmin(red[c][t], red[c][t + h]);
        red[3 + c][t] = fmax(red[3 + c][t], red[3 + c][t + h]);
      }
    __syncthreads();
  }
  if (t < 6) out[t] = red[t][0];
}

// ------------------------------------------------------------------- the step

// timer names of the per-class attention launches (class c covers n in (32c, 32c + 32])
const char *const kAttnFwdName[4] = {"attn_fwd_n32", "attn_fwd_n64", "attn_fwd_n96",
                                     "attn_fwd_n128"};
const char *const kAttnFwdLnName[4] = {"attn_fwd_ln_n32", "attn_fwd_ln_n64", "attn_fwd_ln_n96",
                                       "attn_fwd_ln_n128"};
const char *const kAttnBwdQName[4] = {"attn_bwd_q_n32", "attn_bwd_q_n64", "attn_bwd_q_n96",
                                      "attn_bwd_q_n128"};
const char *const kAttnBwdName[4] = {"attn_bwd_n32", "attn_bwd_n64", "attn_bwd_n96",
                                     "attn_bwd_n128"};
const char *const kAttnBwdKName[4] = {"attn_bwd_k_n32", "attn_bwd_k_n64", "attn_bwd_k_n96",
                                      "attn_bwd_k_n128"};

// The attention forward applies the output projection and layer norm itself
// when the embedding width pads to kAttnOpCols columns and the attention
// width is 128 (the shapes its kernel is built for).
bool attn_fwd_fuses_projection(const dp_model *m) {
  return m->ldM == kAttnOpCols && m->dattn == 128;
}

#define RUN(name, call)                                           \
  do {                                                            \
    hipEvent_t a_ = nullptr, b_ = nullptr;                        \
    if (m->timer.enabled) {                                       \
      a_ = m->timer.get();                                        \
      b_ = m->timer.get();                                        \
      if (a_) (void)hipEventRecord(a_, s);                        \
    }                                                             \
    call;                                                         \
    if (a_ && b_) {                                               \
      (void)hipEventRecord(b_, s);                                \
      m->timer.pending.push_back({name, a_, b_});                 \
    }                                                             \
  } while (0)

// Forward half of the step: neighbour lists through the atomic energies.
// Leaves every activation the adjoint needs in the workspace.
int enqueue_forward(dp_model *m, const double *d_coords, const int32_t *d_types,
                    const CellGrid &grid, int nloc, int nall, double *d_energy,
                    double *d_atom_energy, hipStream_t s) {
  auto &w = m->w;
  const int sel = m->sel;
  const int *Pptr = w.pair_off + nloc;
  const int ne = (int)m->emb.size(), na = m->n_attn, nf = (int)m->fit.size();

  RUN("init", hipLaunchKernelGGL(k_init_step, dim3((grid.ncell + 255) / 256), dim3(256), 0, s,
                                 m->flags, w.ccount, w.cell_count, w.cell_fill, grid.ncell));
  RUN("check_types", launch_check_types(d_types, nall, m->ntypes, m->flags, w.types_safe, s));
  d_types = w.types_safe;
  RUN("cell_bin", launch_cell_bin(d_coords, nall, grid, w.atom_cell, w.cell_count, s));
  RUN("cell_scan", launch_scan(w.cell_count, grid.ncell, w.cell_start, s));
  RUN("cell_fill", launch_cell_fill(w.atom_cell, nall, w.cell_start, w.cell_fill, w.cell_atoms, s));
  RUN("nlist", launch_nlist(d_coords, nloc, nall, grid, m->rcut, sel, w.cell_start, w.cell_atoms,
                            w.nlist, w.nnei, m->flags, s));
  RUN("pair_scan", launch_scan(w.nnei, nloc, w.pair_off, s));
  if (m->cap_pairs < 0 || m->want_pairs > m->cap_pairs || m->cap_pairs_nloc != m->cap_nloc) {
    // lay the pair arena out from this step's pair count (the only blocking
    // point of a step, at the first step of a workspace and after growth)
    int total = 0;
    HIP_TRY(hipMemcpyAsync(&total, w.pair_off + nloc, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int rc = ensure_pairs(m, std::max<long>(total, m->want_pairs));
    if (rc) return rc;
  } else {
    RUN("pair_guard", hipLaunchKernelGGL(k_pair_guard, dim3(1), dim3(1024), 0, s, w.pair_off,
                                         w.nnei, nloc, nall, m->cap_pairs, m->flags));
  }
  const int Pmax = (int)std::min<long>((long)nloc * sel, m->cap_pairs);
  // attention classes to launch: those that held centres in a recent step
  // (the host copy of the counts lags the device by a step or more; a stale
  // choice costs padding, never correctness), always the top one
  const int ncls = attn_class_count(sel);
  int active = (1 << ncls) - 1;
  if (m->ccount_host[4] >= 0) {
    active = 1 << (ncls - 1);
    for (int c = 0; c < ncls - 1; ++c)
      if (m->ccount_host[4 + c] > 0) active |= 1 << c;
    // the largest class with the fused FP32 adjoint stays launched, so that a
    // centre is always computed by the same kind of adjoint (fused or not)
    // and results do not depend on which classes were empty before
    const AttnArgs probe{nullptr, nullptr, nullptr, nullptr, nullptr, nloc, sel, 0.f, m->bf16};
    for (int c = ncls - 2; c >= 0; --c)
      if (attn_bwd_fused(probe, c) && !attn_bwd_fused(probe, ncls - 1)) {
        active |= 1 << c;
        break;
      }
  }
  // the top class is always launched (nothing above it takes its centres);
  // when it held none recently, on a small grid
  int small = 0;
  if (m->ccount_host[4] >= 0 && m->ccount_host[4 + ncls - 1] == 0) small = 1 << (ncls - 1);
  m->cls_active = active;
  m->cls_small = small;
  if (na > 0)
    RUN("attn_classes", launch_attn_classes(w.nnei, nloc, active, w.ccount, w.clist, s));
  RUN("env_embed1",
      launch_env_embed1(d_coords, d_types, grid, nloc, sel, m->rcut, m->rcut_smth, w.nlist,
                        w.nnei, w.pair_off, m->type_table, m->ws, m->ntypes, m->emb[0],
                        m->lde[0], w.geom, w.h[0], s));
  // embedding layers
  const bool emb_fused = ne == 3 && emb_fused_supported(m->lde[0], m->lde[1], m->lde[2]);
  EmbLaunch el{};
  if (emb_fused) {
    el = EmbLaunch{w.h[0], m->embl[1].Wt, m->embl[1].b, m->embl[2].Wt, m->embl[2].b,
                   m->embl[1].Wb, m->embl[2].Wb, m->ws, m->emb[0], m->emb[1], m->emb[2],
                   m->embl[1].res, m->embl[2].res, Pptr, Pmax, m->bf16};
    RUN("emb_fwd", launch_emb_fwd(el, w.h[2], s));
  } else {
    for (int l = 1; l < ne; ++l) {
      const Linear &L = m->embl[l];
      GemmArgs a{w.h[l - 1], L.ldin, L.Wt, L.ldin, L.ldout, L.fout, Pptr, Pmax, m->bf16};
      RUN("emb_fwd", gemm_tanh_res(a, L.b, nullptr, 0, w.h[l - 1], L.ldin, L.res, L.fin, w.h[l],
                                   L.ldout, w.te[l], L.ldout, s));
    }
  }
  // attention layers
  const int D = m->dattn, ldM = m->ldM;
  const AttnArgs aa{w.geom, w.pair_off, w.nnei,       w.clist,      w.ccount,
                    nloc,   sel,        (float)m->shift, m->bf16, m->cls_small};
  for (int a = 0; a < na; ++a) {
    const auto &A = m->attn[a];
    // in BF16 mode QKV, o, dO and dQKV are stored in BF16 (matrix-core operands only)
    GemmArgs g1{w.G[a], ldM, A.Wt_qkv, ldM, 3 * D, 3 * D, Pptr, Pmax, m->bf16, 0, m->M};
    RUN("qkv_fwd", gemm_linear(g1, A.b_qkv, w.qkv[a], 3 * D, s, m->bf16));
    const AttnOut op{A.Wt_o, A.b_o,      A.gamma,   A.beta,    (float)m->ln_eps,
                     w.G[a], w.G[a + 1], w.xhat[a], w.rstd[a], m->M};
    const bool fuse_op = attn_fwd_fuses_projection(m);
    for (int cls = 0; cls < ncls; ++cls)
      if ((active >> cls) & 1)
        RUN(fuse_op ? kAttnFwdLnName[cls] : kAttnFwdName[cls],
            launch_attn_fwd_class(cls, aa, w.qkv[a], w.o[a], w.lam[a], w.fstat[a],
                                  fuse_op ? &op : nullptr, s));
    if (!fuse_op) {
      GemmArgs g2{w.o[a], D, A.Wt_o, D, ldM, m->M, Pptr, Pmax, m->bf16, m->bf16};
      RUN("oproj_ln_fwd", gemm_ln_res(g2, A.b_o, A.gamma, A.beta, (float)m->ln_eps, w.G[a], ldM,
                                      w.G[a + 1], w.xhat[a], w.rstd[a], s));
    }
  }
  // descriptor and fitting
  RUN("desc_fwd", launch_desc_fwd(w.geom, w.G[na], ldM, w.pair_off, w.nnei, nloc, sel, m->M,
                                  m->axis, w.T, w.dmat, s));
  {
    const Linear &L = m->fitl[0];
    GemmArgs a{w.dmat, m->ldD, L.Wt, m->ldD, L.ldout, L.fout, nullptr, nloc, m->bf16};
    // few centres (a small domain): the long-k first layer split over k, with
    // the attention adjoint's dQKV buffer (unused until the adjoint) as scratch
    const size_t scratch = (size_t)(m->cap_pairs + 64) * 3 * std::max(m->dattn, 16);
    RUN("fit_fwd", {
      if (!gemm_tanh_res_split(a, m->fb0, d_types, L.ldout, w.z[0], L.ldout, w.tf[0], L.ldout,
                               w.dqkv, m->cap_pairs >= 0 ? scratch : 0, s))
        gemm_tanh_res(a, m->fb0, d_types, L.ldout, nullptr, 0, RES_NONE, 0, w.z[0], L.ldout,
                      w.tf[0], L.ldout, s);
    });
  }
  for (int l = 1; l < nf; ++l) {
    const Linear &L = m->fitl[l];
    GemmArgs a{w.z[l - 1], L.ldin, L.Wt, L.ldin, L.ldout, L.fout, nullptr, nloc, m->bf16};
    RUN("fit_fwd", gemm_tanh_res(a, L.b, nullptr, 0, w.z[l - 1], L.ldin, L.res, L.fin, w.z[l],
                                 L.ldout, w.tf[l], L.ldout, s));
  }
  RUN("energy", launch_energy(w.z[nf - 1], w.tf[nf - 1], m->ldf[nf - 1], m->fit[nf - 1],
                              m->w_out, m->b_out, m->ebias, d_types, nloc, w.e, w.fa[nf - 1], s));
  if (d_energy)
    RUN("reduce", launch_reduce(w.e, w.vir_part, nloc, d_energy, nullptr, d_atom_energy, s));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(m->flags_host, m->flags, sizeof(DevFlags), hipMemcpyDeviceToHost, s));
  if (na > 0 && nloc > 0)
    HIP_TRY(hipMemcpyAsync(m->ccount_host, w.ccount, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
  m->last = s;
  m->have_step = true;
  m->last_nloc = nloc;
  m->fwd = dp_model::FwdState{d_coords, grid, nloc, nall, true};
  m->shared_layer = na - 1;
  return DP_OK;
}

// Adjoint half: from unit seeds de_i/de_i down to g_ij = de_i/dd_ij, then the
// weighted gather sign * (-sum_i wgt_i de_i/dx_k) and the virial.
int enqueue_backward(dp_model *m, const double *wgt, double sign, double *d_out,
                     double *d_virial, hipStream_t s) {
  auto &w = m->w;
  const dp_model::FwdState &fs = m->fwd;
  const double *d_coords = fs.coords;
  const CellGrid &grid = fs.grid;
  const int nloc = fs.nloc, nall = fs.nall;
  const int sel = m->sel;
  const int Pmax = (int)std::min<long>((long)nloc * sel, m->cap_pairs);
  const int *Pptr = w.pair_off + nloc;
  const int ne = (int)m->emb.size(), na = m->n_attn, nf = (int)m->fit.size();
  const int D = m->dattn, ldM = m->ldM;
  const AttnArgs aa{w.geom, w.pair_off, w.nnei,       w.clist,      w.ccount,
                    nloc,   sel,        (float)m->shift, m->bf16, m->cls_small};
  const bool emb_fused = ne == 3 && emb_fused_supported(m->lde[0], m->lde[1], m->lde[2]);
  EmbLaunch el{};
  if (emb_fused)
    el = EmbLaunch{w.h[0], m->embl[1].Wt, m->embl[1].b, m->embl[2].Wt, m->embl[2].b,
                   m->embl[1].Wb, m->embl[2].Wb, m->ws, m->emb[0], m->emb[1], m->emb[2],
                   m->embl[1].res, m->embl[2].res, Pptr, Pmax, m->bf16};
  // fitting adjoint: fa[l] = dz_l * (1 - t_l^2) ; dz_{l-1} = fa[l] W_l^T + res^T(dz_l)
  for (int l = nf - 1; l >= 1; --l) {
    const Linear &L = m->fitl[l];
    GemmArgs a{w.fa[l], L.ldout, L.Wb, L.ldout, L.ldin, L.fin, nullptr, nloc, m->bf16};
    int mode = RES_NONE;
    const float *res = nullptr;
    if (l == nf - 1) {
      if (L.res == RES_IDENT) {
        mode = RES_BCAST;
        res = m->w_out;
      }
    } else {
      res = w.fdz[l];
      mode = L.res == RES_IDENT ? RES_IDENT : (L.res == RES_DOUBLE ? RES_FOLD : RES_NONE);
    }
    RUN("fit_bwd", gemm_bwd_tanh(a, res, L.ldout, mode, L.fin, w.tf[l - 1], L.ldin, w.fdz[l - 1],
                                 L.ldin, w.fa[l - 1], L.ldin, s));
  }
  {
    const Linear &L = m->fitl[0];
    GemmArgs a{w.fa[0], L.ldout, L.Wb, L.ldout, m->ldD, m->M * m->axis, nullptr, nloc, m->bf16};
    RUN("fit_bwd", gemm_linear(a, nullptr, w.dD, m->ldD, s));
  }
  // descriptor adjoint -> dG of the last layer, plus the next layer-norm / tanh seed
  float *dG_cur = w.dGa, *dG_nxt = w.dGb;
  // (the fused embedding adjoint takes no seed buffer: the modes that would
  // write one are not used then)
  float *emb_du_top = emb_fused ? w.dY : w.du[ne - 1];
  const bool desc_fused = na > 0 && desc_oproj_fusable(ldM, m->M, m->axis, D);
  if (desc_fused) {
    const auto &A = m->attn[na - 1];
    RUN("desc_oproj_bwd",
        launch_desc_oproj_bwd(w.geom, w.G[na], w.T, w.dD, w.pair_off, w.nnei, nloc, sel, m->M,
                              m->axis, A.gamma, w.xhat[na - 1], w.rstd[na - 1], A.Wb_o, dG_cur,
                              w.dRt, w.dO, m->bf16, s));
  } else {
    const int ln_mode = na > 0 ? 0 : (emb_fused ? 2 : 1);
    const float *gam = na > 0 ? m->attn[na - 1].gamma : nullptr;
    const float *xh = na > 0 ? w.xhat[na - 1] : nullptr;
    const float *rs = na > 0 ? w.rstd[na - 1] : nullptr;
    float *dnext = na > 0 ? w.dY : emb_du_top;
    RUN("desc_bwd", launch_desc_bwd(w.geom, w.G[na], ldM, w.T, w.dD, w.pair_off, w.nnei, nloc,
                                    sel, m->M, m->axis, ln_mode, gam, xh, rs, w.te[ne - 1],
                                    dG_cur, dnext, w.dRt, s));
  }
  if (na == 0) {
    RUN("zero_attn_grads", {
      hipLaunchKernelGGL(k_fill_int, dim3((Pmax + 255) / 256), dim3(256), 0, s, (int *)w.gw,
                         Pmax, 0);
      hipLaunchKernelGGL(k_fill_int, dim3((4 * Pmax + 255) / 256), dim3(256), 0, s,
                         (int *)w.gr, 4 * Pmax, 0);
    });
  }
  for (int a = na - 1; a >= 0; --a) {
    const auto &A = m->attn[a];
    if (m->recompute && m->shared_layer != a) {
      // the shared buffers hold another layer: recompute this layer's forward
      // from its stored input G[a] (the same kernels, so the same values)
      GemmArgs r1{w.G[a], ldM, A.Wt_qkv, ldM, 3 * D, 3 * D, Pptr, Pmax, m->bf16, 0, m->M};
      RUN("qkv_fwd_recompute", gemm_linear(r1, A.b_qkv, w.qkv[a], 3 * D, s, m->bf16));
      const AttnOut op{A.Wt_o, A.b_o,      A.gamma,   A.beta,    (float)m->ln_eps,
                       w.G[a], w.G[a + 1], w.xhat[a], w.rstd[a], m->M};
      const bool fuse_op = attn_fwd_fuses_projection(m);
      for (int cls = 0; cls < attn_class_count(sel); ++cls)
        if ((m->cls_active >> cls) & 1)
          RUN("attn_fwd_recompute",
              launch_attn_fwd_class(cls, aa, w.qkv[a], w.o[a], w.lam[a], w.fstat[a],
                                    fuse_op ? &op : nullptr, s));
      if (!fuse_op) {
        GemmArgs r2{w.o[a], D, A.Wt_o, D, ldM, m->M, Pptr, Pmax, m->bf16, m->bf16};
        RUN("oproj_ln_recompute", gemm_ln_res(r2, A.b_o, A.gamma, A.beta, (float)m->ln_eps,
                                              w.G[a], ldM, w.G[a + 1], w.xhat[a], w.rstd[a], s));
      }
      m->shared_layer = a;
    }
    GemmArgs g1{w.dY, ldM, A.Wb_o, ldM, D, D, Pptr, Pmax, m->bf16, 0, m->M};
    if (!(desc_fused && a == na - 1))  // else dO came with the descriptor adjoint
      RUN("oproj_bwd", gemm_linear(g1, nullptr, w.dO, D, s, m->bf16));
    for (int cls = 0; cls < attn_class_count(sel); ++cls)
      if (((m->cls_active >> cls) & 1) && attn_bwd_fused(aa, cls))
        RUN(kAttnBwdName[cls],
          launch_attn_bwd_fused_class(cls, aa, w.qkv[a], w.dO, w.lam[a], w.fstat[a], w.dqkv,
                                      w.gw, w.gr, a != na - 1, s));
    for (int cls = 0; cls < attn_class_count(sel); ++cls)
      if (((m->cls_active >> cls) & 1) && !attn_bwd_fused(aa, cls))
        RUN(kAttnBwdQName[cls],
          launch_attn_bwd_q_class(cls, aa, w.qkv[a], w.o[a], w.dO, w.lam[a], w.fstat[a], w.dqkv,
                                  w.astat, w.qside, w.dA, s));
    for (int cls = 0; cls < attn_class_count(sel); ++cls)
      if (((m->cls_active >> cls) & 1) && !attn_bwd_fused(aa, cls))
        RUN(kAttnBwdKName[cls],
          launch_attn_bwd_k_class(cls, aa, w.qkv[a], w.dO, w.lam[a], w.dA, w.dqkv, w.astat,
                                  w.qside,
                                  w.gw, w.gr, a != na - 1, s));
    GemmArgs g2{w.dqkv, 3 * D, A.Wb_qkv, 3 * D, ldM, m->M, Pptr, Pmax, m->bf16, m->bf16};
    const int mode = a > 0 ? 0 : (emb_fused ? 2 : 1);
    const float *gam = a > 0 ? m->attn[a - 1].gamma : nullptr;
    const float *xh = a > 0 ? w.xhat[a - 1] : nullptr;
    const float *rs = a > 0 ? w.rstd[a - 1] : nullptr;
    float *dnext = a > 0 ? w.dY : emb_du_top;
    RUN("qkv_bwd", gemm_qkv_bwd(g2, dG_cur, mode, gam, xh, rs, w.te[ne - 1], dG_nxt, dnext, s));
    std::swap(dG_cur, dG_nxt);
  }
  // embedding adjoint; dG_cur is dE/dG0 = dE/dh_{ne-1}
  if (emb_fused) RUN("emb_bwd", launch_emb_bwd(el, dG_cur, w.gs, s));
  w.dh[ne - 1] = dG_cur;
  for (int l = ne - 1; l >= 1 && !emb_fused; --l) {
    const Linear &L = m->embl[l];
    GemmArgs a{w.du[l], L.ldout, L.Wb, L.ldout, L.ldin, L.fin, Pptr, Pmax, m->bf16};
    const int mode = L.res == RES_IDENT ? RES_IDENT : (L.res == RES_DOUBLE ? RES_FOLD : RES_NONE);
    if (l >= 2) {
      RUN("emb_bwd", gemm_bwd_tanh(a, w.dh[l], L.ldout, mode, L.fin, w.te[l - 1], L.ldin,
                                   w.dh[l - 1], L.ldin, w.du[l - 1], L.ldin, s));
    } else {
      RUN("emb_bwd", gemm_emb1_bwd(a, w.dh[1], L.ldout, mode, L.fin, w.h[0], L.ldin, m->ws, w.gs,
                                   s));
    }
  }
  RUN("env_bwd", launch_env_bwd(w.geom, w.gs, w.dRt, w.gw, w.gr, Pptr, Pmax, 0.f, w.g, s));
  RUN("forces", launch_forces(d_coords, grid, nloc, nall, sel, w.nlist, w.nnei, w.pair_off, w.g,
                              wgt, sign, d_out, w.vir_part, s));
  if (d_virial)
    RUN("reduce", launch_reduce(w.e, w.vir_part, nloc, nullptr, d_virial, nullptr, s));
  HIP_TRY(hipGetLastError());
  m->last = s;
  return DP_OK;
}

int enqueue_step(dp_model *m, const double *d_coords, const int32_t *d_types, const CellGrid &grid,
                 int nloc, int nall, double *d_energy, double *d_forces, double *d_virial,
                 double *d_atom_energy, hipStream_t s) {
  int rc = enqueue_forward(m, d_coords, d_types, grid, nloc, nall, d_energy, d_atom_energy, s);
  if (rc) return rc;
  return enqueue_backward(m, nullptr, 1.0, d_forces, d_virial, s);
}

int check_flags(dp_model *m) {
  const DevFlags &f = *m->flags_host;
  if (f.pair_overflow > 0) {
    m->want_pairs = f.pair_overflow;
    return fail(DP_ERR_CAPACITY,
                "the step had %d neighbour pairs, more than the %ld the workspace holds; its "
                "outputs are not valid and the workspace grows at the next call",
                f.pair_overflow, m->cap_pairs);
  }
  if (f.bad_type_atom != INT_MAX)
    return fail(DP_ERR_TYPE, "atom %d has a type outside [0, %d)", f.bad_type_atom, m->ntypes);
  if (f.overflow_atom != INT_MAX)
    return fail(DP_ERR_SEL_OVERFLOW, "atom %d has %d neighbours within rcut > sel = %d",
                f.overflow_atom, f.overflow_count, m->sel);
  return DP_OK;
}

int common_checks(dp_model *m, const void *coords, const void *types, int nloc, int nghost,
                  const void *energy, const void *forces, const void *virial) {
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (nloc < 0 || nghost < 0) return fail(DP_ERR_ARG, "nloc and nghost must be >= 0");
  if ((long)nloc + nghost > INT_MAX / 4) return fail(DP_ERR_ARG, "too many atoms");
  if ((long)nloc * m->sel > INT_MAX / 8) return fail(DP_ERR_ARG, "nloc * sel too large");
  const int nall = nloc + nghost;
  if (nall > 0 && (!coords || !types)) return fail(DP_ERR_ARG, "coords/types is NULL");
  if (!energy || !virial || (nall > 0 && !forces))
    return fail(DP_ERR_ARG, "an output pointer is NULL");
  return DP_OK;
}

int set_device(dp_model *m) {
  HIP_TRY(hipSetDevice(m->device));
  return DP_OK;
}

}  // namespace

// ======================================================================= C ABI

extern "C" {

const char *dp_last_error(void) { return g_err.c_str(); }

int dp_create(const char *weights_path, double rcut, int sel, dp_model **out) {
  g_err.clear();
  if (!weights_path || !out) return fail(DP_ERR_ARG, "weights_path/out is NULL");
  *out = nullptr;
  if (!(rcut > 0) || !std::isfinite(rcut)) return fail(DP_ERR_ARG, "rcut must be > 0");
  if (sel < 1 || sel > DP_MAX_SEL) return fail(DP_ERR_ARG, "sel must be in [1, %d]", DP_MAX_SEL);
  // parse the header first so that file errors are reported without a device
  {
    FILE *f = fopen(weights_path, "rb");
    if (!f) return fail(DP_ERR_WEIGHTS, "cannot open weights file '%s'", weights_path);
    char magic[8] = {0};
    const size_t n = fread(magic, 1, 8, f);
    fclose(f);
    if (n != 8 || memcmp(magic, "DPA1WTS\0", 8) != 0)
      return fail(DP_ERR_WEIGHTS, "'%s' is not a DPA-1 weights file", weights_path);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(DP_ERR_DEVICE, "no HIP device available");
  dp_model *m = new dp_model();
  m->rcut = rcut;
  m->sel = sel;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return fail(DP_ERR_DEVICE, "hipGetDevice failed");
  }
  int rc = load_weights(m, weights_path);
  if (rc == DP_OK && !(m->rcut_smth < rcut))
    rc = fail(DP_ERR_ARG, "rcut %g must exceed rcut_smth %g", rcut, m->rcut_smth);
  if (rc == DP_OK) {
    hipError_t e = hipMalloc(&m->flags, sizeof(DevFlags));
    if (e == hipSuccess) e = hipMalloc(&m->bbox, 6 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(&m->flags_host, sizeof(DevFlags));
    if (e == hipSuccess) e = hipHostMalloc(&m->ccount_host, 8 * sizeof(int));
    if (e == hipSuccess) m->ccount_host[4] = -1;  // no counts yet: every class active
    if (e == hipSuccess) e = hipStreamCreate(&m->own);
    if (e == hipSuccess) e = attn_prepare();
    if (e != hipSuccess) rc = fail(DP_ERR_DEVICE, "device setup failed: %s", hipGetErrorString(e));
  }
  if (rc != DP_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return DP_OK;
}

void dp_destroy(dp_model *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->last) (void)hipStreamSynchronize(m->last);
  delete m;
}

int dp_model_info(const dp_model *m, int32_t *ints, double *dbls) {
  if (!m || !ints || !dbls) return fail(DP_ERR_ARG, "NULL argument");
  ints[0] = m->ntypes;
  ints[1] = m->tebd;
  ints[2] = m->axis;
  ints[3] = m->n_attn;
  ints[4] = m->dattn;
  ints[5] = m->M;
  ints[6] = m->fit.back();
  ints[7] = m->sel;
  dbls[0] = m->rcut;
  dbls[1] = m->rcut_smth;
  dbls[2] = m->shift;
  return DP_OK;
}

int dp_compute(dp_model *m, const double *coords, const int32_t *types, const double *box,
               int nloc, int nghost, double *energy, double *forces, double *virial,
               double *atom_energy) {
  g_err.clear();
  int rc = common_checks(m, coords, types, nloc, nghost, energy, forces, virial);
  if (rc) return rc;
  const int nall = nloc + nghost;
  for (int k = 0; k < nall; ++k)
    if (types[k] < 0 || types[k] >= m->ntypes)
      return fail(DP_ERR_TYPE, "atom %d has type %d outside [0, %d)", k, types[k], m->ntypes);
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < 3 * nall; ++k)
    if (!std::isfinite(coords[k])) return fail(DP_ERR_ARG, "coordinate %d is not finite", k);
  if (nall > 0) {
    for (int c = 0; c < 3; ++c) lo[c] = hi[c] = coords[c];
    for (int k = 0; k < nall; ++k)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], coords[3 * k + c]);
        hi[c] = std::max(hi[c], coords[3 * k + c]);
      }
  }
  CellGrid grid;
  if ((rc = make_grid(m, box, lo, hi, grid))) return rc;
  if ((rc = set_device(m))) return rc;
  if ((rc = ensure_workspace(m, nloc, nall, grid.ncell))) return rc;
  hipStream_t s = m->own;
  auto &w = m->w;
  if (nall > 0) {
    HIP_TRY(hipMemcpyAsync(w.coords, coords, sizeof(double) * 3 * nall, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w.types, types, sizeof(int32_t) * nall, hipMemcpyHostToDevice, s));
  }
  if ((rc = enqueue_step(m, w.coords, w.types, grid, nloc, nall, w.out_e, w.out_f, w.out_v,
                         w.out_ae, s)))
    return rc;
  // a step that outgrew the pair arena is run again on the grown arena
  HIP_TRY(hipStreamSynchronize(s));
  if (m->flags_host->pair_overflow > 0) {
    m->want_pairs = m->flags_host->pair_overflow;
    if ((rc = enqueue_step(m, w.coords, w.types, grid, nloc, nall, w.out_e, w.out_f, w.out_v,
                           w.out_ae, s)))
      return rc;
  }
  std::vector<double> F(3 * (size_t)nall), AE(nloc);
  double E = 0, V[9];
  HIP_TRY(hipMemcpyAsync(&E, w.out_e, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(V, w.out_v, sizeof(double) * 9, hipMemcpyDeviceToHost, s));
  if (nall > 0)
    HIP_TRY(hipMemcpyAsync(F.data(), w.out_f, sizeof(double) * 3 * nall, hipMemcpyDeviceToHost, s));
  if (atom_energy && nloc > 0)
    HIP_TRY(hipMemcpyAsync(AE.data(), w.out_ae, sizeof(double) * nloc, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (m->timer.enabled) m->timer.collect();
  if ((rc = check_flags(m))) return rc;
  *energy = E;
  memcpy(virial, V, sizeof(V));
  if (nall > 0) memcpy(forces, F.data(), sizeof(double) * 3 * nall);
  if (atom_energy && nloc > 0) memcpy(atom_energy, AE.data(), sizeof(double) * nloc);
  return DP_OK;
}

int dp_compute_device(dp_model *m, const double *d_coords, const int32_t *d_types,
                      const double *box, int nloc, int nghost, double *d_energy,
                      double *d_forces, double *d_virial, double *d_atom_energy,
                      void *hip_stream) {
  g_err.clear();
  int rc = common_checks(m, d_coords, d_types, nloc, nghost, d_energy, d_forces, d_virial);
  if (rc) return rc;
  const int nall = nloc + nghost;
  if ((rc = set_device(m))) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  if (!box && nall > 0) {
    // open boundaries: the cell grid needs the bounding box of the atoms
    double hb[6];
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(256), 0, s, d_coords, nall, m->bbox);
    HIP_TRY(hipMemcpyAsync(hb, m->bbox, sizeof(hb), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < 3; ++c) {
      lo[c] = hb[c];
      hi[c] = hb[3 + c];
      if (!std::isfinite(lo[c]) || !std::isfinite(hi[c]))
        return fail(DP_ERR_ARG, "coordinates are not finite");
    }
  }
  CellGrid grid;
  if ((rc = make_grid(m, box, lo, hi, grid))) return rc;
  if ((rc = ensure_workspace(m, nloc, nall, grid.ncell))) return rc;
  return enqueue_step(m, d_coords, d_types, grid, nloc, nall, d_energy, d_forces, d_virial,
                      d_atom_energy, s);
}

int dp_forward_device(dp_model *m, const double *d_coords, const int32_t *d_types,
                      const double *box, int nloc, int nghost, double *d_energy,
                      double *d_atom_energy, void *hip_stream) {
  g_err.clear();
  double dummy = 0.0;
  int rc = common_checks(m, d_coords, d_types, nloc, nghost, d_energy, &dummy, &dummy);
  if (rc) return rc;
  const int nall = nloc + nghost;
  if ((rc = set_device(m))) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  if (!box && nall > 0) {
    double hb[6];
    hipLaunchKernelGGL(k_bbox, dim3(1), dim3(256), 0, s, d_coords, nall, m->bbox);
    HIP_TRY(hipMemcpyAsync(hb, m->bbox, sizeof(hb), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < 3; ++c) {
      lo[c] = hb[c];
      hi[c] = hb[3 + c];
      if (!std::isfinite(lo[c]) || !std::isfinite(hi[c]))
        return fail(DP_ERR_ARG, "coordinates are not finite");
    }
  }
  CellGrid grid;
  if ((rc = make_grid(m, box, lo, hi, grid))) return rc;
  if ((rc = ensure_workspace(m, nloc, nall, grid.ncell))) return rc;
  return enqueue_forward(m, d_coords, d_types, grid, nloc, nall, d_energy, d_atom_energy, s);
}

int dp_backward_device(dp_model *m, const double *d_atom_weight, double *d_grad_coords,
                       double *d_virial, void *hip_stream) {
  g_err.clear();
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (!m->fwd.valid) return fail(DP_ERR_ARG, "no forward step to differentiate");
  if (m->fwd.nall > 0 && !d_grad_coords) return fail(DP_ERR_ARG, "d_grad_coords is NULL");
  int rc;
  if ((rc = set_device(m))) return rc;
  return enqueue_backward(m, d_atom_weight, -1.0, d_grad_coords, d_virial,
                          (hipStream_t)hip_stream);
}

int dp_sync(dp_model *m) {
  g_err.clear();
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (!m->have_step) return DP_OK;
  int rc;
  if ((rc = set_device(m))) return rc;
  HIP_TRY(hipStreamSynchronize(m->last));
  if (m->timer.enabled) m->timer.collect();
  return check_flags(m);
}

int dp_debug_nlist(dp_model *m, int32_t *nlist, int32_t *nnei) {
  g_err.clear();
  if (!m || !nlist || !nnei) return fail(DP_ERR_ARG, "NULL argument");
  if (!m->have_step) return fail(DP_ERR_ARG, "no step has been computed");
  int rc;
  if ((rc = set_device(m))) return rc;
  HIP_TRY(hipStreamSynchronize(m->last));
  const int n = m->last_nloc;
  if (n > 0) {
    HIP_TRY(hipMemcpy(nlist, m->w.nlist, sizeof(int32_t) * (size_t)n * m->sel,
                      hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(nnei, m->w.nnei, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  }
  return DP_OK;
}

int dp_set_precision(dp_model *m, int precision) {
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (precision != DP_PREC_FP32 && precision != DP_PREC_BF16)
    return fail(DP_ERR_ARG, "unknown precision %d", precision);
  if (m->last) (void)hipStreamSynchronize(m->last);
  m->bf16 = precision == DP_PREC_BF16;
  m->fwd.valid = false;  // a pending adjoint must come from a forward in the new mode
  return DP_OK;
}

int dp_set_memory_budget(dp_model *m, double bytes) {
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (!(bytes >= 0) || !std::isfinite(bytes)) return fail(DP_ERR_ARG, "bad memory budget");
  if (m->last) (void)hipStreamSynchronize(m->last);
  m->mem_budget = bytes;
  // the layout is chosen again at the next step
  if (m->arena || m->parena) {
    int rc = set_device(m);
    if (rc) return rc;
    if ((rc = free_arenas(m))) return rc;
  }
  return DP_OK;
}

int dp_memory_info(const dp_model *m, int64_t *workspace_bytes, int32_t *recompute) {
  if (!m || !workspace_bytes || !recompute) return fail(DP_ERR_ARG, "NULL argument");
  *workspace_bytes = (int64_t)(m->arena_bytes + m->parena_bytes);
  *recompute = m->recompute ? 1 : 0;
  return DP_OK;
}

int dp_set_timing(dp_model *m, int enable) {
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (m->last) (void)hipStreamSynchronize(m->last);
  m->timer.collect();
  m->timer.enabled = enable != 0;
  m->timer.totals.clear();
  return DP_OK;
}

int dp_kernel_times(dp_model *m, char *names, int64_t *counts, double *total_ms, int max) {
  if (!m) return fail(DP_ERR_ARG, "model handle is NULL");
  if (m->last) (void)hipStreamSynchronize(m->last);
  m->timer.collect();
  int k = 0;
  for (auto &kv : m->timer.totals) {
    if (k < max) {
      if (names) {
        strncpy(names + 48 * k, kv.first.c_str(), 47);
        names[48 * k + 47] = 0;
      }
      if (counts) counts[k] = kv.second.first;
      if (total_ms) total_ms[k] = kv.second.second;
    }
    ++k;
  }
  return k;
}

}  // extern "C"
