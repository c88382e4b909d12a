// Per-centre kernels of DPA-1: the gated neighbour self-attention core and
// the descriptor contraction, forward and input-gradient backward.
//
// DPA-1 refines the embedding matrix G of each centre with gated
// self-attention blocks that act only within that centre's neighbour set
// and whose gate carries the angular term R R^T (Sec. II-B, DPA-1); the
// descriptor is D = G^T R~ R~^T G_< (Sec. II-B, DP-SE).  With the per-pair
// switch w = sw(r) and unit vectors rhat the attention of one centre is
//   lam_qk = q_q . k_k / sqrt(d)
//   L_qk   = (lam_qk + S) w_q w_k - S
//   P_qk   = exp(L_qk) / (sum_k' exp(L_qk') + (sel - n) exp(-S))
//   A_qk   = P_qk w_q w_k (rhat_q . rhat_k)
//   o_q    = sum_k A_qk v_k
// The shift S, the w_q w_k factors and the (sel - n) exp(-S) term make the
// energy continuous when a neighbour crosses the cutoff (sw -> 0 turns its
// logit into -S, the value the padding term stands for).
//
// Layout: one workgroup per centre, one wavefront per 16-neighbour tile
// (n <= 128 -> at most 8 tiles).  All products run on
// v_mfma_f32_16x16x4_f32.  Logit tiles are computed transposed, S^T = K Q^T,
// so that lane l holds keys 4*(l/16)+{0..3} of query l%16: that register
// layout is exactly the B operand of the next product (A V, dS K, ...),
// so probabilities never leave registers in the forward pass.
#include <cfloat>

#include "dpa1_internal.h"

namespace dpa1 {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kMaxTiles = 8;     // 128 neighbours
constexpr int kQKV = 3;          // q, k, v blocks in one row of the projection output

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sum_groups(float v) {  // over lanes sharing lane%16
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ __forceinline__ float max_groups(float v) {
  v = fmaxf(v, __shfl_xor(v, 16));
  v = fmaxf(v, __shfl_xor(v, 32));
  return v;
}
__device__ __forceinline__ float sum_rows(float v) {  // over the 16 lanes of a group
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  return v;
}

// Per-neighbour gate data staged in LDS: (rhat_x, rhat_y, rhat_z, sw), zero
// for slots beyond n.
__device__ __forceinline__ void stage_keys(const float *__restrict__ geom, int base, int n,
                                           float4 *kg) {
  for (int t = threadIdx.x; t < kMaxTiles * 16; t += blockDim.x) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < n) {
      const float *gp = geom + (size_t)(base + t) * kGeom;
      v = make_float4(gp[G_RX], gp[G_RY], gp[G_RZ], gp[G_SW]);
    }
    kg[t] = v;
  }
}

// S^T tile for key tile kt and the wave's query registers qv.
// dattn = 128 = 8 chunks of 16 features.
__device__ __forceinline__ floatx4 qk_tile(const float *__restrict__ rows, int ld, int base,
                                           int n, int kt, int r, int g, const floatx4 (&qv)[8]) {
  floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
  const int key = kt * 16 + r;
  const bool ok = key < n;
  const float *kr = rows + (size_t)(base + (ok ? key : 0)) * ld + 4 * g;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const floatx4 kv = ok ? *(const floatx4 *)(kr + 16 * c) : floatx4{0.f, 0.f, 0.f, 0.f};
    acc = mfma4(kv[0], qv[c][0], acc);
    acc = mfma4(kv[1], qv[c][1], acc);
    acc = mfma4(kv[2], qv[c][2], acc);
    acc = mfma4(kv[3], qv[c][3], acc);
  }
  return acc;
}

// Load one 16x128 row tile as the MFMA B operand: lane holds row r,
// features 16c + 4g + {0..3}.
__device__ __forceinline__ void load_rows(const float *__restrict__ rows, int ld, int base,
                                          int n, int row, int g, floatx4 (&v)[8]) {
  const bool ok = row < n;
  const float *p = rows + (size_t)(base + (ok ? row : 0)) * ld + 4 * g;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    v[c] = ok ? *(const floatx4 *)(p + 16 * c) : floatx4{0.f, 0.f, 0.f, 0.f};
}

// acc[ft] += X^T B for one 16-row tile of X (rows 'tile*16 + 4g + t', all 128
// features) and a 16x16 B tile held as bt (lane: column r, rows 4g + t).
__device__ __forceinline__ void accum_xt_b(const float *__restrict__ rows, int ld, int base,
                                           int n, int tile, int r, int g, const floatx4 &bt,
                                           floatx4 (&acc)[8]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int row = tile * 16 + 4 * g + t;
    const bool ok = row < n;
    const float *p = rows + (size_t)(base + (ok ? row : 0)) * ld + r;
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) {
      const float x = ok ? p[16 * ft] : 0.f;
      acc[ft] = mfma4(x, bt[t], acc[ft]);
    }
  }
}

// --------------------------------------------------------------------- forward

__global__ __launch_bounds__(512) void k_attn_fwd(const float *__restrict__ qkv,
                                                  const float *__restrict__ geom,
                                                  const int *__restrict__ pair_off,
                                                  const int *__restrict__ nnei, int sel,
                                                  float shift, float *__restrict__ out) {
  __shared__ float4 kg[kMaxTiles * 16];
  const int i = blockIdx.x;
  const int n = nnei[i];
  const int base = pair_off[i];
  stage_keys(geom, base, n, kg);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int ntile = (n + 15) >> 4;
  if (wave >= ntile) return;
  const int r = lane & 15, g = lane >> 4;
  const int q = wave * 16 + r;
  const bool qok = q < n;
  const int ld = kQKV * 128;
  const float inv_sqrt_d = 0.08838834764831845f;  // 1/sqrt(128)

  floatx4 qv[8];
  load_rows(qkv, ld, base, n, q, g, qv);
  floatx4 st[kMaxTiles];
#pragma unroll
  for (int kt = 0; kt < kMaxTiles; ++kt)
    if (kt < ntile) st[kt] = qk_tile(qkv + 128, ld, base, n, kt, r, g, qv);

  const float4 gq = kg[q];
  const float wq = qok ? gq.w : 0.f;
  float mx = -FLT_MAX;
#pragma unroll
  for (int kt = 0; kt < kMaxTiles; ++kt) {
    if (kt >= ntile) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = kt * 16 + 4 * g + v;
      const float wk = kg[k].w;
      float l = (st[kt][v] * inv_sqrt_d + shift) * wq * wk - shift;
      l = k < n ? l : -INFINITY;
      st[kt][v] = l;
      mx = fmaxf(mx, l);
    }
  }
  const float m = fmaxf(max_groups(mx), -shift);
  float z = 0.f;
#pragma unroll
  for (int kt = 0; kt < kMaxTiles; ++kt) {
    if (kt >= ntile) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float e = expf(st[kt][v] - m);
      st[kt][v] = e;
      z += e;
    }
  }
  z = sum_groups(z) + (float)(sel - n) * expf(-shift - m);
  const float invz = 1.0f / z;

  floatx4 oacc[8];
#pragma unroll
  for (int ft = 0; ft < 8; ++ft) oacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < kMaxTiles; ++kt) {
    if (kt >= ntile) continue;
    floatx4 at;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float4 gk = kg[kt * 16 + 4 * g + v];
      const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
      at[v] = st[kt][v] * invz * wq * gk.w * c;
    }
    accum_xt_b(qkv + 256, ld, base, n, kt, r, g, at, oacc);
  }
  if (!qok) return;
  float *op = out + (size_t)(base + q) * 128 + 4 * g;
#pragma unroll
  for (int ft = 0; ft < 8; ++ft) *(floatx4 *)(op + 16 * ft) = oacc[ft];
}

// -------------------------------------------------------------------- backward
//
// Given dO, with H = w_q w_k c_qk (c = rhat_q . rhat_k):
//   dA = dO V^T ; dV = A^T dO ; dP = dA H ; dH = dA P
//   D_q = sum_k P dP = dO_q . o_q ; dL = P (dP - D_q)
//   dS = dL w_q w_k / sqrt(d) ; dQ = dS K ; dK = dS^T Q
//   X = dL (lam + S) + dH c  -> dw_q += sum_k X w_k, dw_k += sum_q X w_q
//   Y = dH w_q w_k           -> drhat_q += sum_k Y rhat_k, drhat_k += sum_q Y rhat_q
// Pass 1 (wave = query tile): P, dA, dL, dQ, query-side sums; A and dS go to
// LDS.  Pass 2 (wave = key tile): dK, dV from the LDS tiles, key-side sums.

__global__ __launch_bounds__(512) void k_attn_bwd(
    const float *__restrict__ qkv, const float *__restrict__ o, const float *__restrict__ dO,
    const float *__restrict__ geom, const int *__restrict__ pair_off,
    const int *__restrict__ nnei, int sel, float shift, float *__restrict__ dqkv,
    float *__restrict__ gw, float *__restrict__ gr, int accumulate) {
  extern __shared__ float lds[];
  float4 *kg = (float4 *)lds;                               // [128]
  float4 *qside = kg + kMaxTiles * 16;                      // [128] query-side (dw, dr)
  float4 *kpart = qside + kMaxTiles * 16;                   // [8 waves][128] key-side
  float *tA = (float *)(kpart + kMaxTiles * kMaxTiles * 16);  // [64 tiles][256]
  float *tS = tA + kMaxTiles * kMaxTiles * 256;              // [64 tiles][256]

  const int i = blockIdx.x;
  const int n = nnei[i];
  const int base = pair_off[i];
  stage_keys(geom, base, n, kg);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int ntile = (n + 15) >> 4;
  const int r = lane & 15, g = lane >> 4;
  const int ld = kQKV * 128;
  const float inv_sqrt_d = 0.08838834764831845f;

  if (wave < ntile) {
    const int qt = wave;
    const int q = qt * 16 + r;
    const bool qok = q < n;
    const float4 gq = kg[q];
    const float wq = qok ? gq.w : 0.f;

    floatx4 qv[8];
    load_rows(qkv, ld, base, n, q, g, qv);
    floatx4 st[kMaxTiles];  // lam, then probabilities
#pragma unroll
    for (int kt = 0; kt < kMaxTiles; ++kt)
      if (kt < ntile) st[kt] = qk_tile(qkv + 128, ld, base, n, kt, r, g, qv);

    floatx4 dov[8];
    load_rows(dO, 128, base, n, q, g, dov);
    // D_q = dO_q . o_q
    float dq = 0.f;
    {
      floatx4 ov[8];
      load_rows(o, 128, base, n, q, g, ov);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        dq += dov[c][0] * ov[c][0] + dov[c][1] * ov[c][1] + dov[c][2] * ov[c][2] +
              dov[c][3] * ov[c][3];
      dq = sum_groups(dq);
    }

    floatx4 lam[kMaxTiles];
    float mx = -FLT_MAX;
#pragma unroll
    for (int kt = 0; kt < kMaxTiles; ++kt) {
      if (kt >= ntile) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 16 + 4 * g + v;
        const float wk = kg[k].w;
        const float lm = st[kt][v] * inv_sqrt_d;
        lam[kt][v] = lm;
        float l = (lm + shift) * wq * wk - shift;
        l = k < n ? l : -INFINITY;
        st[kt][v] = l;
        mx = fmaxf(mx, l);
      }
    }
    const float m = fmaxf(max_groups(mx), -shift);
    float z = 0.f;
#pragma unroll
    for (int kt = 0; kt < kMaxTiles; ++kt) {
      if (kt >= ntile) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float e = expf(st[kt][v] - m);
        st[kt][v] = e;
        z += e;
      }
    }
    z = sum_groups(z) + (float)(sel - n) * expf(-shift - m);
    const float invz = 1.0f / z;

    floatx4 dqacc[8];
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) dqacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
    float dwq = 0.f, drqx = 0.f, drqy = 0.f, drqz = 0.f;

#pragma unroll
    for (int kt = 0; kt < kMaxTiles; ++kt) {
      if (kt >= ntile) continue;
      const floatx4 da = qk_tile(qkv + 256, ld, base, n, kt, r, g, dov);  // dA^T tile
      floatx4 at, ds;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 16 + 4 * g + v;
        const float4 gk = kg[k];
        const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
        const float ww = wq * gk.w;
        const float p = qok ? st[kt][v] * invz : 0.f;
        const float h = ww * c;
        const float dP = da[v] * h;
        const float dH = da[v] * p;
        const float dL = p * (dP - dq);
        at[v] = p * h;
        ds[v] = dL * ww * inv_sqrt_d;
        const float X = dL * (lam[kt][v] + shift) + dH * c;
        const float Y = dH * ww;
        dwq += X * gk.w;
        drqx += Y * gk.x;
        drqy += Y * gk.y;
        drqz += Y * gk.z;
        // key side: sum over the 16 queries of this wave
        float kx = sum_rows(X * wq);
        float ky0 = sum_rows(Y * gq.x);
        float ky1 = sum_rows(Y * gq.y);
        float ky2 = sum_rows(Y * gq.z);
        if (r == 0) kpart[qt * (kMaxTiles * 16) + k] = make_float4(kx, ky0, ky1, ky2);
      }
      accum_xt_b(qkv + 128, ld, base, n, kt, r, g, ds, dqacc);
      // A and dS tiles, element (q_local = r, k_local = 4g + v)
      const int tix = (qt * kMaxTiles + kt) * 256 + r * 16 + 4 * g;
      *(floatx4 *)(tA + tix) = at;
      *(floatx4 *)(tS + tix) = ds;
    }
    dwq = sum_groups(dwq);
    drqx = sum_groups(drqx);
    drqy = sum_groups(drqy);
    drqz = sum_groups(drqz);
    if (g == 0) qside[q] = make_float4(dwq, drqx, drqy, drqz);
    if (qok) {
      float *dp = dqkv + (size_t)(base + q) * ld + 4 * g;
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) *(floatx4 *)(dp + 16 * ft) = dqacc[ft];
    }
  }
  __syncthreads();
  if (wave >= ntile) return;

  // pass 2: wave owns key tile kt
  const int kt = wave;
  floatx4 dkacc[8], dvacc[8];
#pragma unroll
  for (int ft = 0; ft < 8; ++ft) {
    dkacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
    dvacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  for (int qt = 0; qt < ntile; ++qt) {
    floatx4 bs, ba;
    const int tb = (qt * kMaxTiles + kt) * 256;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bs[t] = tS[tb + (4 * g + t) * 16 + r];
      ba[t] = tA[tb + (4 * g + t) * 16 + r];
    }
    accum_xt_b(qkv, ld, base, n, qt, r, g, bs, dkacc);
    accum_xt_b(dO, 128, base, n, qt, r, g, ba, dvacc);
  }
  const int key = kt * 16 + r;
  if (key < n) {
    float *dp = dqkv + (size_t)(base + key) * ld + 4 * g;
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) {
      *(floatx4 *)(dp + 128 + 16 * ft) = dkacc[ft];
      *(floatx4 *)(dp + 256 + 16 * ft) = dvacc[ft];
    }
    if (g == 0) {
      float4 tot = qside[key];
      for (int w = 0; w < ntile; ++w) {
        const float4 kp = kpart[w * (kMaxTiles * 16) + key];
        tot.x += kp.x;
        tot.y += kp.y;
        tot.z += kp.z;
        tot.w += kp.w;
      }
      const size_t p = (size_t)(base + key);
      if (accumulate) {
        gw[p] += tot.x;
        gr[4 * p + 0] += tot.y;
        gr[4 * p + 1] += tot.z;
        gr[4 * p + 2] += tot.w;
      } else {
        gw[p] = tot.x;
        gr[4 * p + 0] = tot.y;
        gr[4 * p + 1] = tot.z;
        gr[4 * p + 2] = tot.w;
        gr[4 * p + 3] = 0.f;
      }
    }
  }
}

// ------------------------------------------------------------------ descriptor

// T[c][m] = (1/sel) sum_j R~_j[c] G_j[m];  D[m][a] = sum_c T[c][m] T[c][a].
__global__ __launch_bounds__(128) void k_desc_fwd(const float *__restrict__ geom,
                                                  const float *__restrict__ G, int ldg,
                                                  const int *__restrict__ pair_off,
                                                  const int *__restrict__ nnei, int sel, int M,
                                                  int axis, float *__restrict__ T,
                                                  float *__restrict__ dmat, int ldd) {
  __shared__ float Ts[4][128];
  const int i = blockIdx.x;
  const int n = nnei[i];
  const int base = pair_off[i];
  const int m = threadIdx.x;
  float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f;
  if (m < M) {
    for (int j = 0; j < n; ++j) {
      const float *gp = geom + (size_t)(base + j) * kGeom;
      const float s = gp[G_S];
      const float gm = G[(size_t)(base + j) * ldg + m];
      t0 += s * gm;
      t1 += s * gp[G_RX] * gm;
      t2 += s * gp[G_RY] * gm;
      t3 += s * gp[G_RZ] * gm;
    }
    const float inv = 1.0f / (float)sel;
    t0 *= inv;
    t1 *= inv;
    t2 *= inv;
    t3 *= inv;
    float *tp = T + (size_t)i * 4 * M;
    tp[m] = t0;
    tp[M + m] = t1;
    tp[2 * M + m] = t2;
    tp[3 * M + m] = t3;
  }
  Ts[0][m] = t0;
  Ts[1][m] = t1;
  Ts[2][m] = t2;
  Ts[3][m] = t3;
  __syncthreads();
  if (m < M) {
    float *dp = dmat + (size_t)i * ldd + (size_t)m * axis;
    for (int a = 0; a < axis; ++a)
      dp[a] = t0 * Ts[0][a] + t1 * Ts[1][a] + t2 * Ts[2][a] + t3 * Ts[3][a];
  }
  // zero the row padding of the descriptor matrix
  for (int c = M * axis + m; c < ldd; c += blockDim.x) dmat[(size_t)i * ldd + c] = 0.f;
}

// dT[c][m] = sum_a dD[m][a] T[c][a] + [m < axis] sum_m' dD[m'][m] T[c][m'];
// per pair: dG_j = (1/sel) R~_j dT, dR~_j = (1/sel) dT G_j, then the
// layer-norm backward of the last attention layer (ln_mode 0) or the tanh
// backward of the last embedding layer (ln_mode 1).
__global__ __launch_bounds__(256) void k_desc_bwd(
    const float *__restrict__ geom, const float *__restrict__ G, int ldg,
    const float *__restrict__ T, const float *__restrict__ dD, int ldd,
    const int *__restrict__ pair_off, const int *__restrict__ nnei, int sel, int M, int axis,
    int ln_mode, const float *__restrict__ gamma, const float *__restrict__ xhat,
    const float *__restrict__ rstd, const float *__restrict__ temb, float *__restrict__ dG,
    float *__restrict__ dnext, float *__restrict__ dRt) {
  __shared__ float Ts[4][128];
  __shared__ float dTs[4][128];
  const int i = blockIdx.x;
  const int n = nnei[i];
  const int base = pair_off[i];
  const int tid = threadIdx.x;
  if (tid < 128) {
    for (int c = 0; c < 4; ++c) Ts[c][tid] = tid < M ? T[(size_t)i * 4 * M + c * M + tid] : 0.f;
  }
  __syncthreads();
  const float inv = 1.0f / (float)sel;
  if (tid < M) {
    const float *dr = dD + (size_t)i * ldd;
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
    for (int a = 0; a < axis; ++a) {
      const float x = dr[tid * axis + a];
      d0 += x * Ts[0][a];
      d1 += x * Ts[1][a];
      d2 += x * Ts[2][a];
      d3 += x * Ts[3][a];
    }
    if (tid < axis) {
      for (int mm = 0; mm < M; ++mm) {
        const float x = dr[mm * axis + tid];
        d0 += x * Ts[0][mm];
        d1 += x * Ts[1][mm];
        d2 += x * Ts[2][mm];
        d3 += x * Ts[3][mm];
      }
    }
    dTs[0][tid] = d0 * inv;
    dTs[1][tid] = d1 * inv;
    dTs[2][tid] = d2 * inv;
    dTs[3][tid] = d3 * inv;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const float invm = 1.0f / (float)M;
  for (int j = wave; j < n; j += 4) {
    const size_t p = (size_t)(base + j);
    const float *gp = geom + p * kGeom;
    const float s = gp[G_S];
    const float R0 = s, R1 = s * gp[G_RX], R2 = s * gp[G_RY], R3 = s * gp[G_RZ];
    float dg[2], xh[2];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = lane + 64 * h;
      dg[h] = 0.f;
      xh[h] = 0.f;
      if (m < M) {
        const float gm = G[p * ldg + m];
        const float v = R0 * dTs[0][m] + R1 * dTs[1][m] + R2 * dTs[2][m] + R3 * dTs[3][m];
        dg[h] = v;
        a0 += gm * dTs[0][m];
        a1 += gm * dTs[1][m];
        a2 += gm * dTs[2][m];
        a3 += gm * dTs[3][m];
        if (ln_mode == 0) {
          xh[h] = xhat[p * ldg + m];
          const float dx = gamma[m] * v;
          s1 += dx;
          s2 += dx * xh[h];
        }
      }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
      a3 += __shfl_xor(a3, off);
      s1 += __shfl_xor(s1, off);
      s2 += __shfl_xor(s2, off);
    }
    const float rs = ln_mode == 0 ? rstd[p] : 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = lane + 64 * h;
      if (m < ldg) {
        float nx = 0.f;
        if (m < M) {
          if (ln_mode == 0) {
            nx = rs * (gamma[m] * dg[h] - s1 * invm - xh[h] * s2 * invm);
          } else {
            const float t = temb[p * ldg + m];
            nx = dg[h] * (1.0f - t * t);
          }
        }
        dG[p * ldg + m] = dg[h];
        dnext[p * ldg + m] = nx;
      }
    }
    if (lane == 0) {
      float *dp = dRt + 4 * p;
      dp[0] = a0;
      dp[1] = a1;
      dp[2] = a2;
      dp[3] = a3;
    }
  }
}

}  // namespace

void launch_attn_fwd(const float *qkv, const float *geom, const int *pair_off, const int *nnei,
                     int nloc, int sel, int dattn, float shift, float *out, hipStream_t s) {
  (void)dattn;
  if (nloc <= 0) return;
  hipLaunchKernelGGL(k_attn_fwd, dim3(nloc), dim3(512), 0, s, qkv, geom, pair_off, nnei, sel,
                     shift, out);
}

size_t attn_bwd_lds_bytes() {
  return sizeof(float4) * (kMaxTiles * 16 * 2 + kMaxTiles * kMaxTiles * 16) +
         sizeof(float) * 2 * kMaxTiles * kMaxTiles * 256;
}

hipError_t set_attn_bwd_lds_limit() {
  return hipFuncSetAttribute((const void *)k_attn_bwd,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)attn_bwd_lds_bytes());
}

void launch_attn_bwd(const float *qkv, const float *o, const float *dO, const float *geom,
                     const int *pair_off, const int *nnei, int nloc, int sel, int dattn,
                     float shift, float *dqkv, float *gw, float *gr, int accumulate,
                     hipStream_t s) {
  (void)dattn;
  if (nloc <= 0) return;
  hipLaunchKernelGGL(k_attn_bwd, dim3(nloc), dim3(512), attn_bwd_lds_bytes(), s, qkv, o, dO,
                     geom, pair_off, nnei, sel, shift, dqkv, gw, gr, accumulate);
}

void launch_desc_fwd(const float *geom, const float *G, int ldg, const int *pair_off,
                     const int *nnei, int nloc, int sel, int M, int axis, float *T, float *dmat,
                     hipStream_t s) {
  if (nloc <= 0) return;
  const int ldd = pad16(M * axis);
  hipLaunchKernelGGL(k_desc_fwd, dim3(nloc), dim3(128), 0, s, geom, G, ldg, pair_off, nnei, sel,
                     M, axis, T, dmat, ldd);
}

void launch_desc_bwd(const float *geom, const float *G, int ldg, const float *T,
                     const float *dD, const int *pair_off, const int *nnei, int nloc, int sel,
                     int M, int axis, int ln_mode, const float *gamma, const float *xhat,
                     const float *rstd, const float *t_emb, float *dG, float *dnext,
                     float *dRt, hipStream_t s) {
  if (nloc <= 0) return;
  const int ldd = pad16(M * axis);
  hipLaunchKernelGGL(k_desc_bwd, dim3(nloc), dim3(256), 0, s, geom, G, ldg, T, dD, ldd,
                     pair_off, nnei, sel, M, axis, ln_mode, gamma, xhat, rstd, t_emb, dG, dnext,
                     dRt);
}

}  // namespace dpa1
