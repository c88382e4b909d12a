// Student-training kernels: loss seeds, the tangent pass along the force
// residual, the reverse sweep through the descriptor and the embedding net,
// weight-gradient reductions and Adam.
//
// Notation (per pair p of centre i): s = sw(r)/r, rhat = d/r,
// R~ = (s, s rhat) (Sec. II-B), G = emb(s; t_j, t_i) with G' = dG/ds,
// T_i = (1/sel) sum_p R~_p (x) G_p, D_i = T^T T[:, :axis] (Sec. II-B DP-SE
// descriptor).  A dot marks the derivative along the displacement field
// Delta (d-dot_p = Delta_j - Delta_i), a bar the adjoint of
// Psi = sum_i (a e_i - e-dot_i).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dpa1_internal.h"
#include "train_internal.h"

namespace dpa1 {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;          // centres per 256-thread block
constexpr int kGS = kTrN3 + 1;     // LDS row stride of per-pair G rows

// Weights are read through the constant address space: the loads are then
// scalar (uniform, never written by the kernel) and the weights live in SGPRs.
typedef const float __attribute__((address_space(4))) *cfp;
__device__ __forceinline__ float wc(const float *p, int i) { return ((cfp)p)[i]; }

__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
}

// ---------------------------------------------------------------- seeds

__global__ __launch_bounds__(256) void k_tr_seed(const double *__restrict__ F,
                                                 const double *__restrict__ Flab, int n, float cf,
                                                 float4 *__restrict__ delta,
                                                 double *__restrict__ sq_part) {
  __shared__ double red[256];
  const int k = blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (k < n) {
    const double dx = F[3 * k] - Flab[3 * k];
    const double dy = F[3 * k + 1] - Flab[3 * k + 1];
    const double dz = F[3 * k + 2] - Flab[3 * k + 2];
    sq = dx * dx + dy * dy + dz * dz;
    delta[k] = make_float4((float)(cf * dx), (float)(cf * dy), (float)(cf * dz), 0.f);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sq_part[blockIdx.x] = red[0];
}

__global__ void k_tr_energy_seed(const double *__restrict__ E, const double *__restrict__ Elab,
                                 double ca, double cl, float *__restrict__ a,
                                 double *__restrict__ le) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double d = E[0] - Elab[0];
    a[0] = (float)(ca * d);
    le[0] = cl * d * d;
  }
}

// ------------------------------------------------------- per-pair helpers

struct PairTangent {
  float s, sdot;
  float Rt[4], Rd[4];  // R~ and its derivative along Delta
};

// Geometry record -> R~, its tangent and s-dot (ds/dr = dsw/r - s/r).
__device__ __forceinline__ PairTangent pair_tangent(const float4 g0, const float4 g1,
                                                    const float4 di, const float4 dj) {
  PairTangent t;
  const float s = g0.x, rx = g0.y, ry = g0.z, rz = g0.w, r = g1.y, dsw = g1.z;
  const float ddx = dj.x - di.x, ddy = dj.y - di.y, ddz = dj.z - di.z;
  const float rdot = rx * ddx + ry * ddy + rz * ddz;
  const float inv_r = 1.0f / r;
  const float sdot = (dsw - s) * inv_r * rdot;
  const float ux = (ddx - rx * rdot) * inv_r, uy = (ddy - ry * rdot) * inv_r,
              uz = (ddz - rz * rdot) * inv_r;
  t.s = s;
  t.sdot = sdot;
  t.Rt[0] = s;
  t.Rt[1] = s * rx;
  t.Rt[2] = s * ry;
  t.Rt[3] = s * rz;
  t.Rd[0] = sdot;
  t.Rd[1] = sdot * rx + s * ux;
  t.Rd[2] = sdot * ry + s * uy;
  t.Rd[3] = sdot * rz + s * uz;
  return t;
}

// First layer h1 = tanh(table[t_j][t_i] + ws s) and h1' = (1 - h1^2) ws.
__device__ __forceinline__ void emb_l1(const TrainPairArgs &a, int tj, int ti, float s,
                                       float h1[kTrN1], float h1d[kTrN1]) {
  const float4 *tab = (const float4 *)(a.table + (size_t)(tj * a.ntypes + ti) * kTrN1);
#pragma unroll
  for (int q = 0; q < kTrN1 / 4; ++q) {
    const float4 tv = tab[q];
    const float zz[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = 4 * q + u;
      const float t = tanh_fast(fmaf(wc(a.ws, o), s, zz[u]));
      h1[o] = t;
      h1d[o] = (1.0f - t * t) * wc(a.ws, o);
    }
  }
}

// Second layer (doubling residual): h2 = tanh(W2^T h1 + b2) + [h1, h1] and its
// derivative h2' = (1 - t^2) W2^T h1' + [h1', h1'].
__device__ __forceinline__ void emb_l2(const TrainPairArgs &a, const float h1[kTrN1],
                                       const float h1d[kTrN1], float h2[kTrN2],
                                       float h2d[kTrN2]) {
#pragma unroll
  for (int o = 0; o < kTrN2; ++o) {
    float z = wc(a.b2, o), zd = 0.f;
#pragma unroll
    for (int k = 0; k < kTrN1; ++k) {
      z = fmaf(wc(a.W2t, o * kTrN1 + k), h1[k], z);
      zd = fmaf(wc(a.W2t, o * kTrN1 + k), h1d[k], zd);
    }
    const float t = tanh_fast(z);
    h2[o] = t + h1[o % kTrN1];
    h2d[o] = (1.0f - t * t) * zd + h1d[o % kTrN1];
  }
}

// Number of 64-pair chunks the block must run: the largest of its centres.
__device__ __forceinline__ int block_chunks(const int *nnei, int nloc) {
  int mx = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int i = blockIdx.x * kWaves + w;
    mx = max(mx, i < nloc ? nnei[i] : 0);
  }
  return (mx + 63) / 64;
}

// ------------------------------------------------------------ tangent pass

// One wave per centre.  Lanes over pairs compute G, G' (embedding forward
// and its s-derivative) and the coefficients of
// T-dot[c][m] = (1/sel) sum_p (R~-dot_p[c] G_p[m] + R~_p[c] s-dot_p G'_p[m]);
// lanes over m then accumulate T-dot and form
// D-dot[m][a] = sum_c (T-dot[c][m] T[c][a] + T[c][m] T-dot[c][a]).
__global__ __launch_bounds__(256) void k_tr_tangent(TrainPairArgs a,
                                                    const float4 *__restrict__ delta,
                                                    float *__restrict__ Td,
                                                    float *__restrict__ Xd, int ldD) {
  __shared__ float sG[kWaves][64 * kGS];
  __shared__ float sGp[kWaves][64 * kGS];
  __shared__ float sC[kWaves][64 * 8];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + w;
  const bool live = i < a.nloc;
  const int ic = live ? i : 0;
  const int n = live ? a.nnei[ic] : 0;
  const int off = a.pair_off[ic];
  const int ti = a.types[ic];
  const float4 di = delta[ic];
  const int nch = block_chunks(a.nnei, a.nloc);
  float tacc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < nch; ++ch) {
    const int p = ch * 64 + lane;
    const bool valid = p < n;
    const int pc = valid ? p : 0;
    const int q = off + pc;
    const float4 *gp = (const float4 *)(a.geom + (size_t)q * kGeom);
    const float4 g0 = gp[0], g1 = gp[1];
    const int j = a.nlist[(size_t)ic * a.sel + pc];
    const int tj = a.types[j];
    const float4 dj = delta[j];
    if (valid) {
      const PairTangent pt = pair_tangent(g0, g1, di, dj);
      float h1[kTrN1], h1d[kTrN1], h2[kTrN2], h2d[kTrN2];
      emb_l1(a, tj, ti, pt.s, h1, h1d);
      emb_l2(a, h1, h1d, h2, h2d);
#pragma unroll 4
      for (int o = 0; o < kTrN3; ++o) {
        float z = wc(a.b3, o), zd = 0.f;
#pragma unroll
        for (int k = 0; k < kTrN2; ++k) {
          z = fmaf(wc(a.W3t, o * kTrN2 + k), h2[k], z);
          zd = fmaf(wc(a.W3t, o * kTrN2 + k), h2d[k], zd);
        }
        const float t = tanh_fast(z);
        sG[w][lane * kGS + o] = t + h2[o % kTrN2];
        sGp[w][lane * kGS + o] = (1.0f - t * t) * zd + h2d[o % kTrN2];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sC[w][lane * 8 + c] = pt.Rd[c] * a.inv_sel;
        sC[w][lane * 8 + 4 + c] = pt.Rt[c] * pt.sdot * a.inv_sel;
      }
    }
    lds_fence();
    const int cnt = max(0, min(64, n - ch * 64));
    for (int pp = 0; pp < cnt; ++pp) {
      const float g = sG[w][pp * kGS + lane], gd = sGp[w][pp * kGS + lane];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        tacc[c] = fmaf(sC[w][pp * 8 + c], g, fmaf(sC[w][pp * 8 + 4 + c], gd, tacc[c]));
    }
    lds_fence();
  }
  // D-dot from T-dot and T (lane = m)
  float tv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    tv[c] = a.T[((size_t)ic * 4 + c) * kTrN3 + lane];
    sC[w][c * 64 + lane] = tv[c];
    sC[w][256 + c * 64 + lane] = tacc[c];
  }
  lds_fence();
  if (live) {
#pragma unroll
    for (int c = 0; c < 4; ++c) Td[((size_t)i * 4 + c) * kTrN3 + lane] = tacc[c];
    float *xp = Xd + (size_t)i * ldD + (size_t)lane * a.axis;
    for (int ax = 0; ax < a.axis; ++ax) {
      float v = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        v = fmaf(tacc[c], sC[w][c * 64 + ax], fmaf(tv[c], sC[w][256 + c * 64 + ax], v));
      xp[ax] = v;
    }
  }
}

// ------------------------------------------------------------ fitting steps

// Top fitting layer (identity residual): y2 = t2 + y1, y2-dot = g2 z2-dot + y1-dot,
// seeds y2-bar = a w, y2-dot-bar = -w.  Writes z2-bar (rows [0, nloc)),
// z2-dot-bar (rows [nloc, 2 nloc)) and a y2 - y2-dot (for w_out).
__global__ void k_tr_fit_top(const float *__restrict__ t2, const float *__restrict__ y2,
                             const float *__restrict__ yd1, const float *__restrict__ zd2,
                             const float *__restrict__ w_out, const float *__restrict__ a,
                             int nloc, int H, int ld, float *__restrict__ zb2,
                             float *__restrict__ wo_rows) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)nloc * ld) return;
  const int o = (int)(k % ld);
  const float av = a[0];
  if (o >= H) {
    zb2[k] = 0.f;
    zb2[k + (size_t)nloc * ld] = 0.f;
    wo_rows[k] = 0.f;
    return;
  }
  const float t = t2[k], g = 1.0f - t * t, w = w_out[o], zd = zd2[k];
  const float yd2 = fmaf(g, zd, yd1[k]);
  zb2[k] = g * (av * w + 2.0f * t * zd * w);
  zb2[k + (size_t)nloc * ld] = -g * w;
  wo_rows[k] = av * y2[k] - yd2;
}

// First fitting layer (tanh, no residual): from y1-bar = yb1 + a w and
// y1-dot-bar = yb1' - w (the residual seeds of the top layer).
__global__ void k_tr_fit_l0(const float *__restrict__ t1, const float *__restrict__ zd1,
                            const float *__restrict__ yb1, const float *__restrict__ w_out,
                            const float *__restrict__ a, int nloc, int H, int ld,
                            float *__restrict__ zb1) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)nloc * ld) return;
  const int o = (int)(k % ld);
  if (o >= H) {
    zb1[k] = 0.f;
    zb1[k + (size_t)nloc * ld] = 0.f;
    return;
  }
  const float w = w_out[o];
  const float t = t1[k], g = 1.0f - t * t;
  const float ybar = yb1[k] + a[0] * w;
  const float ydbar = yb1[k + (size_t)nloc * ld] - w;
  const float gbar = zd1[k] * ydbar;
  zb1[k] = g * (ybar - 2.0f * t * gbar);
  zb1[k + (size_t)nloc * ld] = g * ydbar;
}

// ------------------------------------------------------------- pair reverse

// One wave per centre.  Lanes over m form T-bar and T-dot-bar from D-bar and
// D-dot-bar (reverse of D = T^T T<, D-dot = T-dot^T T< + T^T T-dot<); lanes
// over pairs then form G-bar = (1/sel)(R~ T-bar + R~-dot T-dot-bar) and
// G'-bar = (1/sel) s-dot R~ T-dot-bar and run the reverse of the embedding net
// and of its s-derivative, writing the rows of the weight gradients.
__global__ __launch_bounds__(256) void k_tr_pair_rev(
    TrainPairArgs a, const float4 *__restrict__ delta, const float *__restrict__ Td,
    const float *__restrict__ Db, int ldD, size_t Pcap, size_t ldr, float *__restrict__ X3,
    float *__restrict__ Z3, float *__restrict__ HB2, int *__restrict__ grp) {
  __shared__ float sT[kWaves][4 * 64], sTd[kWaves][4 * 64];
  __shared__ float sDb[kWaves][64 * 16], sDdb[kWaves][64 * 16];
  __shared__ float sTb[kWaves][4 * 64], sTdb[kWaves][4 * 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + w;
  const bool live = i < a.nloc;
  const int ic = live ? i : 0;
  const int n = live ? a.nnei[ic] : 0;
  const int off = a.pair_off[ic];
  const int ti = a.types[ic];
  const int ax = a.axis;
  const int nloc = a.nloc;
  // --- T-bar, T-dot-bar (lane = m)
  float tv[4], tdv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    tv[c] = a.T[((size_t)ic * 4 + c) * kTrN3 + lane];
    tdv[c] = Td[((size_t)ic * 4 + c) * kTrN3 + lane];
    sT[w][c * 64 + lane] = tv[c];
    sTd[w][c * 64 + lane] = tdv[c];
  }
  for (int b = 0; b < ax; ++b) {
    sDb[w][lane * 16 + b] = Db[(size_t)ic * ldD + (size_t)lane * ax + b];
    sDdb[w][lane * 16 + b] = Db[(size_t)(nloc + ic) * ldD + (size_t)lane * ax + b];
  }
  lds_fence();
  float tb[4] = {0.f, 0.f, 0.f, 0.f}, tdb[4] = {0.f, 0.f, 0.f, 0.f};
  for (int b = 0; b < ax; ++b) {
    const float db = sDb[w][lane * 16 + b], ddb = sDdb[w][lane * 16 + b];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      tb[c] = fmaf(db, sT[w][c * 64 + b], fmaf(ddb, sTd[w][c * 64 + b], tb[c]));
      tdb[c] = fmaf(ddb, sT[w][c * 64 + b], tdb[c]);
    }
  }
  if (lane < ax) {
    for (int mp = 0; mp < kTrN3; ++mp) {
      const float db = sDb[w][mp * 16 + lane], ddb = sDdb[w][mp * 16 + lane];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        tb[c] = fmaf(db, sT[w][c * 64 + mp], fmaf(ddb, sTd[w][c * 64 + mp], tb[c]));
        tdb[c] = fmaf(ddb, sT[w][c * 64 + mp], tdb[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    sTb[w][c * 64 + lane] = tb[c] * a.inv_sel;
    sTdb[w][c * 64 + lane] = tdb[c] * a.inv_sel;
  }
  lds_fence();
  // --- pairs
  const float4 di = delta[ic];
  const unsigned ld32 = (unsigned)ldr, pc32 = (unsigned)Pcap;
  const int nch = block_chunks(a.nnei, a.nloc);
  for (int ch = 0; ch < nch; ++ch) {
    const int p = ch * 64 + lane;
    const bool valid = p < n;
    const int pc = valid ? p : 0;
    const size_t q = (size_t)off + pc;
    const float4 *gp = (const float4 *)(a.geom + q * kGeom);
    const float4 g0 = gp[0], g1 = gp[1];
    const int j = a.nlist[(size_t)ic * a.sel + pc];
    const int tj = a.types[j];
    const float4 dj = delta[j];
    if (!valid) continue;
    const PairTangent pt = pair_tangent(g0, g1, di, dj);
    float h1[kTrN1], h1d[kTrN1], h2[kTrN2], h2d[kTrN2];
    emb_l1(a, tj, ti, pt.s, h1, h1d);
    emb_l2(a, h1, h1d, h2, h2d);
    // feature-major stores: 32-bit offsets advanced one feature row at a time
    // (the host keeps 64 * ldr below 2^32)
    {
      unsigned off = (unsigned)q;
#pragma unroll
      for (int k = 0; k < kTrN2; ++k) {
        X3[off] = h2[k];
        X3[off + pc32] = h2d[k];
        off += ld32;
      }
    }
    // third layer (doubling residual) in reverse
    float hb2[kTrN2], hb2d[kTrN2];
#pragma unroll
    for (int k = 0; k < kTrN2; ++k) hb2[k] = hb2d[k] = 0.f;
    unsigned zoff = (unsigned)q;
#pragma unroll 1
    for (int o = 0; o < kTrN3; ++o) {
      float Gb = 0.f, Gdb = 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float b1v = sTb[w][c * 64 + o], b2v = sTdb[w][c * 64 + o];
        Gb = fmaf(pt.Rt[c], b1v, fmaf(pt.Rd[c], b2v, Gb));
        Gdb = fmaf(pt.Rt[c], b2v, Gdb);
      }
      Gdb *= pt.sdot;
      float z = wc(a.b3, o), zd = 0.f;
#pragma unroll
      for (int k = 0; k < kTrN2; ++k) {
        z = fmaf(wc(a.W3t, o * kTrN2 + k), h2[k], z);
        zd = fmaf(wc(a.W3t, o * kTrN2 + k), h2d[k], zd);
      }
      const float t = tanh_fast(z), g = 1.0f - t * t;
      const float zbd = g * Gdb;
      const float zb = g * (Gb - 2.0f * t * zd * Gdb);
#pragma unroll
      for (int k = 0; k < kTrN2; ++k) {
        hb2[k] = fmaf(wc(a.W3t, o * kTrN2 + k), zb, hb2[k]);
        hb2d[k] = fmaf(wc(a.W3t, o * kTrN2 + k), zbd, hb2d[k]);
      }
      Z3[zoff] = zb;
      Z3[zoff + pc32] = zbd;
      zoff += ld32;
    }
    // the [h2, h2] residual: G-bar[k] and G-bar[k + 32] both feed h2[k]
#pragma unroll
    for (int k = 0; k < kTrN2; ++k) {
      float gb = 0.f, gdb = 0.f;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int o = k + hh * kTrN2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float b1v = sTb[w][c * 64 + o], b2v = sTdb[w][c * 64 + o];
          gb = fmaf(pt.Rt[c], b1v, fmaf(pt.Rd[c], b2v, gb));
          gdb = fmaf(pt.Rt[c], b2v, gdb);
        }
      }
      hb2[k] += gb;
      hb2d[k] = fmaf(gdb, pt.sdot, hb2d[k]);
    }
    {
      unsigned off = (unsigned)q;
#pragma unroll
      for (int k = 0; k < kTrN2; ++k) {
        HB2[off] = hb2[k];
        HB2[off + pc32] = hb2d[k];
        off += ld32;
      }
    }
    grp[q] = tj * a.ntypes + ti;
  }
}


// Second and first embedding layers in reverse, one lane per pair (flat over
// the pair rows): from h2-bar, h2'-bar of the per-centre sweep, recomputing
// h1, h1' from s and the pair's types.
__global__ __launch_bounds__(256) void k_tr_pair_rev2(TrainPairArgs a, const int *__restrict__ Pdev,
                                                      size_t Pcap, size_t ldr,
                                                      const float *__restrict__ HB2,
                                                      const int *__restrict__ grp,
                                                      float *__restrict__ X2, float *__restrict__ Z2,
                                                      float *__restrict__ Z1,
                                                      float *__restrict__ WS1) {
  const int P = Pdev[0];
  const unsigned ld32 = (unsigned)ldr, pc32 = (unsigned)Pcap;
  for (int qi = blockIdx.x * 256 + threadIdx.x; qi < P; qi += gridDim.x * 256) {
    const unsigned q = (unsigned)qi;
    const float s = a.geom[(size_t)q * kGeom + G_S];
    const int g = grp[q];
    const int tj = g / a.ntypes, ti = g - tj * a.ntypes;
    float hb2[kTrN2], hb2d[kTrN2];
    {
      unsigned off = q;
#pragma unroll
      for (int k = 0; k < kTrN2; ++k) {
        hb2[k] = HB2[off];
        hb2d[k] = HB2[off + pc32];
        off += ld32;
      }
    }
    float h1[kTrN1], h1d[kTrN1];
    emb_l1(a, tj, ti, s, h1, h1d);
    {
      unsigned off = q;
#pragma unroll
      for (int k = 0; k < kTrN1; ++k) {
        X2[off] = h1[k];
        X2[off + pc32] = h1d[k];
        off += ld32;
      }
    }
    const PairTangent pt{s};
    // second layer (doubling residual) in reverse
    float hb1[kTrN1], hb1d[kTrN1];
#pragma unroll
    for (int k = 0; k < kTrN1; ++k) hb1[k] = hb1d[k] = 0.f;
#pragma unroll
    for (int o4 = 0; o4 < kTrN2; o4 += 4) {
      float zbv[4], zbdv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = o4 + u;
        float z = wc(a.b2, o), zd = 0.f;
#pragma unroll
        for (int k = 0; k < kTrN1; ++k) {
          z = fmaf(wc(a.W2t, o * kTrN1 + k), h1[k], z);
          zd = fmaf(wc(a.W2t, o * kTrN1 + k), h1d[k], zd);
        }
        const float t = tanh_fast(z), g = 1.0f - t * t;
        const float zbd = g * hb2d[o];
        const float zb = g * (hb2[o] - 2.0f * t * zd * hb2d[o]);
#pragma unroll
        for (int k = 0; k < kTrN1; ++k) {
          hb1[k] = fmaf(wc(a.W2t, o * kTrN1 + k), zb, hb1[k]);
          hb1d[k] = fmaf(wc(a.W2t, o * kTrN1 + k), zbd, hb1d[k]);
        }
        hb1[o % kTrN1] += hb2[o];
        hb1d[o % kTrN1] += hb2d[o];
        zbv[u] = zb;
        zbdv[u] = zbd;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned off = (unsigned)(o4 + u) * ld32 + (unsigned)q;
        Z2[off] = zbv[u];
        Z2[off + pc32] = zbdv[u];
      }
    }
    // first layer: h1' = (1 - h1^2) ws
#pragma unroll
    for (int o4 = 0; o4 < kTrN1; o4 += 4) {
      float zbv[4], wsv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = o4 + u;
        const float g = 1.0f - h1[o] * h1[o];
        const float gbar = wc(a.ws, o) * hb1d[o];
        const float zb = g * (hb1[o] - 2.0f * h1[o] * gbar);
        zbv[u] = zb;
        wsv[u] = fmaf(pt.s, zb, g * hb1d[o]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned off = (unsigned)(o4 + u) * ld32 + (unsigned)q;
        Z1[off] = zbv[u];
        WS1[off] = wsv[u];
      }
    }
  }
}

// ------------------------------------------------------- weight gradients

// part[blk][kin_pad][nout_pad] = sum over the block's rows of X^T Z for both
// segments.  Block = 4 waves over one 16KT x 16NT output tile group; each
// wave takes every 4th group of rows, the four waves are summed in LDS.
// ONEHOT: the X operand is not read but generated, X[r][k] = (group[r] == k)
// (group == nullptr: X[r][k] = (k == 0)), so the product sums Z by group.
template <int KT, int NT, bool BF, bool ONEHOT>
__global__ __launch_bounds__(256) void k_wgrad(const float *__restrict__ X1,
                                               const float *__restrict__ X2, int ldx,
                                               const float *__restrict__ Z1,
                                               const float *__restrict__ Z2, int ldz, int kin,
                                               int nout, const int *__restrict__ rows_dev,
                                               int rows_max, int rows_per_block,
                                               const int32_t *__restrict__ group,
                                               float *__restrict__ part, int kin_pad,
                                               int nout_pad) {
  __shared__ float red[4][KT * NT * 256];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rows = rows_dev ? min(rows_dev[0], rows_max) : rows_max;
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = min(rows, r0 + rows_per_block);
  const int k0 = blockIdx.y * 16 * KT, n0 = blockIdx.z * 16 * NT;
  floatx4 acc[KT][NT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[kt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int col = lane & 15, quad = lane >> 4;
  constexpr int RG = BF ? 32 : 4;  // rows per matrix-core step
  const int nseg = (ONEHOT || X2 == nullptr) ? 1 : 2;
  for (int seg = 0; seg < nseg; ++seg) {
    const float *X = seg ? X2 : X1;
    const float *Z = seg ? Z2 : Z1;
    for (int rg = r0 + w * RG; rg < r1; rg += 4 * RG) {
      if constexpr (!BF) {
        const int r = rg + quad;
        const bool rv = r < r1;
        const size_t rr = (size_t)(rv ? r : r0);
        float xv[KT], zv[NT];
        if constexpr (ONEHOT) {
          const int gr = group ? group[rr] : 0;
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) xv[kt] = (rv && gr == k0 + 16 * kt + col) ? 1.f : 0.f;
        } else {
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const int c = k0 + 16 * kt + col;
            const float v = X[rr * ldx + (c < kin ? c : 0)];
            xv[kt] = (rv && c < kin) ? v : 0.f;
          }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int c = n0 + 16 * nt + col;
          const float v = Z[rr * ldz + (c < nout ? c : 0)];
          zv[nt] = (rv && c < nout) ? v : 0.f;
        }
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[kt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[kt], zv[nt], acc[kt][nt], 0, 0, 0);
      } else {
        // 32 rows per 16x16x32 step: lane slots u < 4 hold rows rg + 4q + u,
        // slots 4 + u rows rg + 16 + 4q + u (the same rows on both operands)
        static_assert(!ONEHOT, "group sums use FP32 operands");
        floatx8 xv[KT], zv[NT];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = rg + 16 * (u >> 2) + 4 * quad + (u & 3);
          const bool rv = r < r1;
          const size_t rr = (size_t)(rv ? r : r0);
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const int c = k0 + 16 * kt + col;
            const float v = X[rr * ldx + (c < kin ? c : 0)];
            xv[kt][u] = (rv && c < kin) ? v : 0.f;
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int c = n0 + 16 * nt + col;
            const float v = Z[rr * ldz + (c < nout ? c : 0)];
            zv[nt][u] = (rv && c < nout) ? v : 0.f;
          }
        }
        bf16x8 xb[KT], zb[NT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) xb[kt] = __builtin_convertvector(xv[kt], bf16x8);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) zb[nt] = __builtin_convertvector(zv[nt], bf16x8);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[kt][nt] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[kt], zb[nt], acc[kt][nt], 0, 0, 0);
      }
    }
  }
  // D[i][j]: register v of lane l holds i = 4 (l / 16) + v, j = l % 16
#pragma unroll
  for (int kt = 0; kt < KT; ++kt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][((kt * NT + nt) * 4 + v) * 64 + lane] = acc[kt][nt][v];
  __syncthreads();
  for (int e = threadIdx.x; e < KT * NT * 256; e += 256) {
    const float sum = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    const int l = e & 63, v = (e >> 6) & 3, tile = e >> 8;
    const int kt = tile / NT, nt = tile % NT;
    const int ki = k0 + 16 * kt + 4 * (l >> 4) + v, nj = n0 + 16 * nt + (l & 15);
    if (ki < kin_pad && nj < nout_pad)
      part[((size_t)blockIdx.x * kin_pad + ki) * nout_pad + nj] = sum;
  }
}

// Feature-major variant: Xt [kin][ldr], Zt [nout][ldr] hold one feature per
// row and the pair rows along it; segment 2 (if seg2 > 0) starts at column
// seg2.  Lane (c, q) of a 16-row step reads rows 4q..4q+3 of feature c as one
// float4, which is the k-slice layout of the BF16 product; the FP32 product
// takes the four components as four 16x16x4 steps.
template <int KT, int NT, bool BF, bool ONEHOT>
__global__ __launch_bounds__(256) void k_wgrad_fm(const float *__restrict__ Xt,
                                                  const float *__restrict__ Zt, size_t ldr,
                                                  size_t seg2, int kin, int nout,
                                                  const int *__restrict__ rows_dev, int rows_max,
                                                  int rows_per_block,
                                                  const int32_t *__restrict__ group,
                                                  float *__restrict__ part, int kin_pad,
                                                  int nout_pad) {
  __shared__ float red[4][KT * NT * 256];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rows = rows_dev ? min(rows_dev[0], rows_max) : rows_max;
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = min(rows, r0 + rows_per_block);
  const int k0 = blockIdx.y * 16 * KT, n0 = blockIdx.z * 16 * NT;
  floatx4 acc[KT][NT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[kt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int col = lane & 15, quad = lane >> 4;
  const int nseg = (ONEHOT || seg2 == 0) ? 1 : 2;
  for (int seg = 0; seg < nseg; ++seg) {
    const size_t base = seg ? seg2 : 0;
    if constexpr (BF) {
      // BF16: 32 rows per gfx950 16x16x32 step; lane slots 0..3 hold rows
      // rg + 4q + 0..3 and slots 4..7 rows rg + 16 + 4q + 0..3, on both
      // operands.  A second half that starts past r1 re-reads the first
      // half's rows (masked to zero).
      static_assert(!ONEHOT, "group sums use FP32 operands");
      for (int rg = r0 + w * 32; rg < r1; rg += 128) {
        const int rq0 = rg + 4 * quad, rq1 = rq0 + 16;
        const int rq1a = rq1 < r1 ? rq1 : rq0;
        bool rv[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          rv[j] = rq0 + j < r1;
          rv[4 + j] = rq1 + j < r1;
        }
        floatx8 xv[KT], zv[NT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int c = k0 + 16 * kt + col;
          const float *xp = Xt + (size_t)(c < kin ? c : 0) * ldr + base;
          const floatx4 v0 = *(const floatx4 *)(xp + rq0), v1 = *(const floatx4 *)(xp + rq1a);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            xv[kt][j] = (rv[j] && c < kin) ? v0[j] : 0.f;
            xv[kt][4 + j] = (rv[4 + j] && c < kin) ? v1[j] : 0.f;
          }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int c = n0 + 16 * nt + col;
          const float *zp = Zt + (size_t)(c < nout ? c : 0) * ldr + base;
          const floatx4 v0 = *(const floatx4 *)(zp + rq0), v1 = *(const floatx4 *)(zp + rq1a);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            zv[nt][j] = (rv[j] && c < nout) ? v0[j] : 0.f;
            zv[nt][4 + j] = (rv[4 + j] && c < nout) ? v1[j] : 0.f;
          }
        }
        bf16x8 xb[KT], zb[NT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) xb[kt] = __builtin_convertvector(xv[kt], bf16x8);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) zb[nt] = __builtin_convertvector(zv[nt], bf16x8);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[kt][nt] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb[kt], zb[nt], acc[kt][nt], 0, 0, 0);
      }
      continue;
    }
    for (int rg = r0 + w * 16; rg < r1; rg += 64) {
      const int rq = rg + 4 * quad;
      bool rv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) rv[j] = rq + j < r1;
      floatx4 xv[KT], zv[NT];
      if constexpr (ONEHOT) {
        const int4 gq = group ? *(const int4 *)(group + rq) : make_int4(0, 0, 0, 0);
        const int gg[4] = {gq.x, gq.y, gq.z, gq.w};
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int j = 0; j < 4; ++j) xv[kt][j] = (rv[j] && gg[j] == k0 + 16 * kt + col) ? 1.f : 0.f;
      } else {
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int c = k0 + 16 * kt + col;
          const floatx4 v = *(const floatx4 *)(Xt + (size_t)(c < kin ? c : 0) * ldr + base + rq);
#pragma unroll
          for (int j = 0; j < 4; ++j) xv[kt][j] = (rv[j] && c < kin) ? v[j] : 0.f;
        }
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = n0 + 16 * nt + col;
        const floatx4 v = *(const floatx4 *)(Zt + (size_t)(c < nout ? c : 0) * ldr + base + rq);
#pragma unroll
        for (int j = 0; j < 4; ++j) zv[nt][j] = (rv[j] && c < nout) ? v[j] : 0.f;
      }
      {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int kt = 0; kt < KT; ++kt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[kt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[kt][j], zv[nt][j],
                                                                  acc[kt][nt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int kt = 0; kt < KT; ++kt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][((kt * NT + nt) * 4 + v) * 64 + lane] = acc[kt][nt][v];
  __syncthreads();
  for (int e = threadIdx.x; e < KT * NT * 256; e += 256) {
    const float sum = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    const int l = e & 63, v = (e >> 6) & 3, tile = e >> 8;
    const int kt = tile / NT, nt = tile % NT;
    const int ki = k0 + 16 * kt + 4 * (l >> 4) + v, nj = n0 + 16 * nt + (l & 15);
    if (ki < kin_pad && nj < nout_pad)
      part[((size_t)blockIdx.x * kin_pad + ki) * nout_pad + nj] = sum;
  }
}

// acc[k][n] += sum_b part[b][k][n] in a fixed order: thread (slice, e) sums
// the blocks b = slice (mod 16) of output e in FP64, then the 16 slices are
// added in slice order.
__global__ __launch_bounds__(256) void k_reduce_parts(const float *__restrict__ part, int nblk,
                                                      int kin_pad, int nout_pad, int kin,
                                                      int nout, double *__restrict__ acc) {
  __shared__ double red[16][16];
  const int el = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int e = blockIdx.x * 16 + el;
  const bool ok = e < kin * nout;
  const int k = ok ? e / nout : 0, n = ok ? e % nout : 0;
  double s = 0.0;
  for (int b = sl; b < nblk; b += 16) s += (double)part[((size_t)b * kin_pad + k) * nout_pad + n];
  red[sl][el] = s;
  __syncthreads();
  if (sl == 0 && ok) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q][el];
    acc[e] += t;
  }
}

// --------------------------------------------------------------------- Adam

__global__ void k_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                       const double *__restrict__ g, int n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = (float)g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  theta[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
}

__global__ void k_fill_f64(double *p, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.0;
}

__global__ __launch_bounds__(256) void k_force_error(const double *__restrict__ a,
                                                     const double *__restrict__ b, int n,
                                                     double *__restrict__ part) {
  __shared__ double ss[256], mx[256];
  double sq = 0.0, m = 0.0;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < 3 * n; k += gridDim.x * 256) {
    const double d = a[k] - b[k];
    sq += d * d;
    m = fmax(m, fabs(d));
  }
  ss[threadIdx.x] = sq;
  mx[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ss[0];
    part[2 * blockIdx.x + 1] = mx[0];
  }
}

inline unsigned nblk(size_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int KT, int NT, bool ONEHOT>
void wgrad_t(const float *X1, const float *X2, int ldx, const float *Z1, const float *Z2, int ldz,
             int kin, int nout, const int *rows_dev, int rows_max, int bf16,
             const int32_t *group, float *part, size_t part_cap, double *acc, hipStream_t s) {
  const int kin_pad = (kin + 15) / 16 * 16, nout_pad = (nout + 15) / 16 * 16;
  const int gy = (kin + 16 * KT - 1) / (16 * KT), gz = (nout + 16 * NT - 1) / (16 * NT);
  const size_t per = (size_t)kin_pad * nout_pad;
  // about two row blocks per compute unit, each a multiple of 64 rows
  int rpb = std::max(1024, (rows_max + 511) / 512);
  rpb = (rpb + 63) / 64 * 64;
  while ((size_t)((rows_max + rpb - 1) / rpb) * per > part_cap) rpb *= 2;
  const int gx = std::max(1, (rows_max + rpb - 1) / rpb);
  const dim3 grid(gx, gy, gz);
  if (bf16 && !ONEHOT)
    hipLaunchKernelGGL((k_wgrad<KT, NT, true, false>), grid, dim3(256), 0, s, X1, X2, ldx, Z1, Z2,
                       ldz, kin, nout, rows_dev, rows_max, rpb, group, part, kin_pad, nout_pad);
  else
    hipLaunchKernelGGL((k_wgrad<KT, NT, false, ONEHOT>), grid, dim3(256), 0, s, X1, X2, ldx, Z1,
                       Z2, ldz, kin, nout, rows_dev, rows_max, rpb, group, part, kin_pad,
                       nout_pad);
  hipLaunchKernelGGL(k_reduce_parts, dim3(nblk((size_t)kin * nout, 16)), dim3(256), 0, s, part,
                     gx, kin_pad, nout_pad, kin, nout, acc);
}

template <int KT, int NT, bool ONEHOT>
void wgrad_fm_t(const float *Xt, const float *Zt, size_t ldr, size_t seg2, int kin, int nout,
                const int *rows_dev, int rows_max, int bf16, const int32_t *group, float *part,
                size_t part_cap, double *acc, hipStream_t s) {
  const int kin_pad = (kin + 15) / 16 * 16, nout_pad = (nout + 15) / 16 * 16;
  const int gy = (kin + 16 * KT - 1) / (16 * KT), gz = (nout + 16 * NT - 1) / (16 * NT);
  const size_t per = (size_t)kin_pad * nout_pad;
  // row blocks of a multiple of 64 rows, about four per compute unit
  int rpb = std::max(512, (rows_max + 1023) / 1024);
  rpb = (rpb + 63) / 64 * 64;
  while ((size_t)((rows_max + rpb - 1) / rpb) * per > part_cap) rpb *= 2;
  const int gx = std::max(1, (rows_max + rpb - 1) / rpb);
  const dim3 grid(gx, gy, gz);
  if (bf16 && !ONEHOT)
    hipLaunchKernelGGL((k_wgrad_fm<KT, NT, true, false>), grid, dim3(256), 0, s, Xt, Zt, ldr,
                       seg2, kin, nout, rows_dev, rows_max, rpb, group, part, kin_pad, nout_pad);
  else
    hipLaunchKernelGGL((k_wgrad_fm<KT, NT, false, ONEHOT>), grid, dim3(256), 0, s, Xt, Zt, ldr,
                       seg2, kin, nout, rows_dev, rows_max, rpb, group, part, kin_pad, nout_pad);
  hipLaunchKernelGGL(k_reduce_parts, dim3(nblk((size_t)kin * nout, 16)), dim3(256), 0, s, part,
                     gx, kin_pad, nout_pad, kin, nout, acc);
}

}  // namespace

int tr_seed_blocks(int n) { return (int)nblk(std::max(n, 1), 256); }

void launch_tr_seed(const double *F, const double *Flab, int n, float cf, float4 *delta,
                    double *sq_part, hipStream_t s) {
  hipLaunchKernelGGL(k_tr_seed, dim3(tr_seed_blocks(n)), dim3(256), 0, s, F, Flab, n, cf, delta,
                     sq_part);
}

void launch_tr_energy_seed(const double *E, const double *Elab, double ca, double cl, float *a,
                           double *le, hipStream_t s) {
  hipLaunchKernelGGL(k_tr_energy_seed, dim3(1), dim3(64), 0, s, E, Elab, ca, cl, a, le);
}

void launch_tr_tangent(const TrainPairArgs &a, const float4 *delta, float *Td, float *Xd, int ldD,
                       hipStream_t s) {
  if (a.nloc <= 0) return;
  hipLaunchKernelGGL(k_tr_tangent, dim3(nblk(a.nloc, kWaves)), dim3(256), 0, s, a, delta, Td, Xd,
                     ldD);
}

void launch_tr_fit_top(const float *t2, const float *y2, const float *yd1, const float *zd2,
                       const float *w_out, const float *a, int nloc, int H, int ld, float *zb2,
                       float *wo_rows, hipStream_t s) {
  const size_t n = (size_t)nloc * ld;
  if (!n) return;
  hipLaunchKernelGGL(k_tr_fit_top, dim3(nblk(n, 256)), dim3(256), 0, s, t2, y2, yd1, zd2, w_out,
                     a, nloc, H, ld, zb2, wo_rows);
}

void launch_tr_fit_l0(const float *t1, const float *zd1, const float *yb1, const float *w_out,
                      const float *a, int nloc, int H, int ld, float *zb1, hipStream_t s) {
  const size_t n = (size_t)nloc * ld;
  if (!n) return;
  hipLaunchKernelGGL(k_tr_fit_l0, dim3(nblk(n, 256)), dim3(256), 0, s, t1, zd1, yb1, w_out, a,
                     nloc, H, ld, zb1);
}

void launch_tr_pair_rev(const TrainPairArgs &a, const float4 *delta, const float *Td,
                        const float *Db, int ldD, size_t Pcap, size_t ldr, float *X3, float *Z3,
                        float *X2, float *Z2, float *Z1, float *WS1, float *HB2, int *grp,
                        hipStream_t s) {
  if (a.nloc <= 0) return;
  hipLaunchKernelGGL(k_tr_pair_rev, dim3(nblk(a.nloc, kWaves)), dim3(256), 0, s, a, delta, Td, Db,
                     ldD, Pcap, ldr, X3, Z3, HB2, grp);
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned blocks = std::min<unsigned>(nblk((size_t)a.nloc * a.sel, 256), 8u * cus);
  hipLaunchKernelGGL(k_tr_pair_rev2, dim3(blocks), dim3(256), 0, s, a, a.pair_off + a.nloc, Pcap,
                     ldr, HB2, grp, X2, Z2, Z1, WS1);
}

void tr_wgrad(const float *X1, const float *X2, int ldx, const float *Z1, const float *Z2, int ldz,
              int kin, int nout, const int *rows_dev, int rows_max, int bf16, float *part,
              size_t part_cap, double *acc, hipStream_t s) {
  if (rows_max <= 0) return;
  if (kin <= 16 && nout <= 32)
    wgrad_t<1, 2, false>(X1, X2, ldx, Z1, Z2, ldz, kin, nout, rows_dev, rows_max, bf16, nullptr,
                         part, part_cap, acc, s);
  else if (kin <= 32 && nout <= 64)
    wgrad_t<2, 4, false>(X1, X2, ldx, Z1, Z2, ldz, kin, nout, rows_dev, rows_max, bf16, nullptr,
                         part, part_cap, acc, s);
  else
    wgrad_t<4, 4, false>(X1, X2, ldx, Z1, Z2, ldz, kin, nout, rows_dev, rows_max, bf16, nullptr,
                         part, part_cap, acc, s);
}

void tr_wgrad_fm(const float *Xt, const float *Zt, size_t ldr, size_t seg2, int kin, int nout,
                 const int *rows_dev, int rows_max, int bf16, float *part, size_t part_cap,
                 double *acc, hipStream_t s) {
  if (rows_max <= 0) return;
  if (kin <= 16 && nout <= 32)
    wgrad_fm_t<1, 2, false>(Xt, Zt, ldr, seg2, kin, nout, rows_dev, rows_max, bf16, nullptr,
                            part, part_cap, acc, s);
  else
    wgrad_fm_t<2, 4, false>(Xt, Zt, ldr, seg2, kin, nout, rows_dev, rows_max, bf16, nullptr,
                            part, part_cap, acc, s);
}

void tr_colsum_fm(const float *Zt, size_t ldr, int ncol, const int *rows_dev, int rows_max,
                  const int32_t *group, int ngroups, float *part, size_t part_cap, double *acc,
                  hipStream_t s) {
  if (rows_max <= 0) return;
  if (ngroups <= 16)
    wgrad_fm_t<1, 4, true>(nullptr, Zt, ldr, 0, ngroups, ncol, rows_dev, rows_max, 0, group, part,
                           part_cap, acc, s);
  else
    wgrad_fm_t<4, 4, true>(nullptr, Zt, ldr, 0, ngroups, ncol, rows_dev, rows_max, 0, group, part,
                           part_cap, acc, s);
}

void tr_colsum(const float *Z, int ldz, int ncol, const int *rows_dev, int rows_max,
               const int32_t *group, int ngroups, float *part, size_t part_cap, double *acc,
               hipStream_t s) {
  if (rows_max <= 0) return;
  if (ngroups <= 16)
    wgrad_t<1, 4, true>(nullptr, nullptr, 0, Z, nullptr, ldz, ngroups, ncol, rows_dev, rows_max,
                        0, group, part, part_cap, acc, s);
  else
    wgrad_t<4, 4, true>(nullptr, nullptr, 0, Z, nullptr, ldz, ngroups, ncol, rows_dev, rows_max,
                        0, group, part, part_cap, acc, s);
}

void launch_adam(float *theta, float *m, float *v, const double *g, int n, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, s, theta, m, v, g, n, lr, b1, b2,
                     eps, bc1, bc2);
}

int force_error_blocks(int n) { return (int)std::min<unsigned>(256, nblk(3 * (size_t)std::max(n, 1), 256)); }

void launch_force_error(const double *a, const double *b, int n, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_force_error, dim3(force_error_blocks(n)), dim3(256), 0, s, a, b, n, part);
}

void launch_fill_f64(double *p, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_f64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n);
}

}  // namespace dpa1
