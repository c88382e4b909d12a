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

// Load one 16x128 row tile as the MFMA B operand: lane holds row r,
// features 16c + 4g + {0..3}.
__device__ __forceinline__ void load_rows(const float *__restrict__ rows, int ld, int base,
                                          int n, int row, int g, floatx4 (&v)[8]) {
  const bool ok = row < n;
  const float *rb = rows + (size_t)base * ld;
  const int off = (ok ? row : 0) * ld + 4 * g;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const floatx4 x = *(const floatx4 *)(rb + off + 16 * c);
    v[c] = ok ? x : floatx4{0.f, 0.f, 0.f, 0.f};
  }
}

// Stage rows [base, base + n) x 128 features of src (row stride ld) into LDS
// transposed, XT[f][k] with row stride NPAD + 4; rows n..NPAD-1 are zero.
// Products that contract over neighbours read it with one 16-byte LDS load
// per lane per four MFMA steps.
template <int NPAD>
__device__ __forceinline__ void stage_t(const float *__restrict__ src, int ld, int base, int n,
                                        float *XT) {
  constexpr int LDT = NPAD + 4;
  constexpr int THREADS = NPAD / 16 * 64;
  constexpr int ITER = NPAD * 32 / THREADS;  // = 8
  float4 v[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int idx = threadIdx.x + it * THREADS;
    const int row = idx >> 5, c4 = idx & 31;
    const int rr = row < n ? row : 0;
    v[it] = *(const float4 *)(src + (size_t)(base + rr) * ld + 4 * c4);
    if (row >= n) v[it] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int idx = threadIdx.x + it * THREADS;
    const int row = idx >> 5, c4 = idx & 31;
    float *d = XT + (4 * c4) * LDT + row;
    d[0] = v[it].x;
    d[LDT] = v[it].y;
    d[2 * LDT] = v[it].z;
    d[3 * LDT] = v[it].w;
  }
}

template <int NPAD>
__device__ __forceinline__ void stage_gate(const float *__restrict__ geom, int base, int n,
                                           float4 *kg) {
  for (int t = threadIdx.x; t < NPAD; t += blockDim.x) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < n) {
      const float *gp = geom + (size_t)(base + t) * kGeom;
      v = make_float4(gp[G_RX], gp[G_RY], gp[G_RZ], gp[G_SW]);
    }
    kg[t] = v;
  }
}

// acc[ft] += XT^T-tile x bt : contraction over the 16 rows of tile 'tile',
// XT in LDS (feature-major), bt a 16x16 B operand held in registers.
template <int NPAD>
__device__ __forceinline__ void accum_lds(const float *XT, int tile, int r, int g,
                                          const floatx4 &bt, floatx4 (&acc)[8]) {
  constexpr int LDT = NPAD + 4;
  floatx4 x[8];
#pragma unroll
  for (int ft = 0; ft < 8; ++ft)
    x[ft] = *(const floatx4 *)(XT + (ft * 16 + r) * LDT + tile * 16 + 4 * g);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) acc[ft] = mfma4(x[ft][t], bt[t], acc[ft]);
}

// Keeps the compiler from hoisting the loads of later iterations (which
// would hold many more registers live than the pipeline needs).
#define SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

// S^T tiles for every key tile: st[kt] (lane: query r, keys 4g + v) from the
// wave's 16 query rows qv and the key rows read from global memory.  The key
// rows of feature chunk c+1 are loaded while chunk c is multiplied.
template <int NT>
__device__ __forceinline__ void qk_tiles(const float *__restrict__ krows, int ld, int base, int n,
                                         int ntile, int r, int g, const floatx4 (&qv)[8],
                                         floatx4 (&st)[NT]) {
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) st[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
  // rows past n read row 0 of the centre and are replaced by zeros; the row
  // base is uniform, per-lane offsets are 32-bit
  const float *kb = krows + (size_t)base * ld;
  int ko[NT];
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
    const int row = kt * 16 + r;
    ko[kt] = (row < n ? row : 0) * ld + 4 * g;
  }
  auto load = [&](int c, floatx4 (&kv)[NT]) {
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
      const floatx4 x = *(const floatx4 *)(kb + ko[kt] + 16 * c);
      kv[kt] = kt * 16 + r < n ? x : floatx4{0.f, 0.f, 0.f, 0.f};
    }
  };
  floatx4 cur[NT], nxt[NT];
  load(0, cur);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c + 1 < 8) load(c + 1, nxt);
    SCHED_FENCE();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) st[kt] = mfma4(cur[kt][t], qv[c][t], st[kt]);
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) cur[kt] = nxt[kt];
  }
}

// One 16x16 tile of rows x kreg^T: lane (row r of the 16-row tile at 'row0',
// lane group g) supplies the A operand from global memory, breg the B operand.
__device__ __forceinline__ floatx4 rows_times(const float *__restrict__ rows, int ld, int base,
                                              int n, int row0, int r, int g,
                                              const floatx4 (&breg)[8]) {
  const int row = row0 + r;
  const bool ok = row < n;
  const float *p = rows + (size_t)(base + (ok ? row : 0)) * ld + 4 * g;
  const floatx4 zero = floatx4{0.f, 0.f, 0.f, 0.f};
  floatx4 a0 = zero, a1 = zero;
  floatx4 x0 = *(const floatx4 *)(p);
  x0 = ok ? x0 : zero;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    floatx4 x1 = zero;
    if (c + 1 < 8) {
      x1 = *(const floatx4 *)(p + 16 * (c + 1));
      x1 = ok ? x1 : zero;
    }
    SCHED_FENCE();
    if (c & 1) {
#pragma unroll
      for (int t = 0; t < 4; ++t) a1 = mfma4(x0[t], breg[c][t], a1);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) a0 = mfma4(x0[t], breg[c][t], a0);
    }
    x0 = x1;
  }
  return a0 + a1;
}

// --------------------------------------------------------------------- forward
//
// One workgroup per centre whose neighbour count lies in (nlo, NPAD]; one
// wavefront per 16-query tile.  V is staged transposed in LDS for A V.

template <int NPAD>
__global__ __launch_bounds__(NPAD / 16 * 64, NPAD <= 64 ? 4 : (NPAD <= 96 ? 3 : 2)) void k_attn_fwd(
    const float *__restrict__ qkv, const float *__restrict__ geom,
    const int *__restrict__ pair_off, const int *__restrict__ nnei, int sel, float shift,
    float *__restrict__ out, int nlo) {
  constexpr int NT = NPAD / 16;
  extern __shared__ float4 smem[];
  float4 *kg = smem;
  float *VT = (float *)(smem + NPAD);
  const int i = blockIdx.x;
  const int n = nnei[i];
  if (n <= nlo || n > NPAD) return;  // uniform over the block
  const int base = pair_off[i];
  const int ntile = (n + 15) >> 4;
  const int ld = kQKV * 128;
  stage_gate<NPAD>(geom, base, n, kg);
  stage_t<NPAD>(qkv + 256, ld, base, n, VT);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= ntile) return;
  const int r = lane & 15, g = lane >> 4;
  const int q = wave * 16 + r;
  const bool qok = q < n;
  const float inv_sqrt_d = 0.08838834764831845f;  // 1/sqrt(128)

  floatx4 qv[8];
  load_rows(qkv, ld, base, n, q, g, qv);
  floatx4 st[NT];
  qk_tiles<NT>(qkv + 128, ld, base, n, ntile, r, g, qv, st);

  const float4 gq = kg[q];
  const float wq = qok ? gq.w : 0.f;
  float mx = -FLT_MAX;
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = kt * 16 + 4 * g + v;
      float l = (st[kt][v] * inv_sqrt_d + shift) * wq * kg[k].w - shift;
      l = k < n ? l : -INFINITY;
      st[kt][v] = l;
      mx = fmaxf(mx, l);
    }
  }
  const float m = fmaxf(max_groups(mx), -shift);
  float z = 0.f;
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
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
  for (int kt = 0; kt < NT; ++kt) {
    floatx4 at;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float4 gk = kg[kt * 16 + 4 * g + v];
      const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
      at[v] = st[kt][v] * invz * wq * gk.w * c;
    }
    accum_lds<NPAD>(VT, kt, r, g, at, oacc);
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
// Phase A (wave = query tile): logits, softmax statistics, dA, dS, dQ and the
// query-side sums (K^T in LDS).  Phase B1 (wave = key tile): logits and dA
// recomputed in the key-major layout, dK and the key-side sums (Q^T in LDS);
// the tile of A is kept in registers for phase B2: dV (dO^T in LDS).

// Backward, in two kernels per class.  k_attn_bwd_q (wave = query tile):
// logits, softmax statistics, dA, dS, dQ and the query-side sums (K^T in
// LDS); it writes the statistics (m, 1/Z, D_q) and the query-side sums per
// pair.  k_attn_bwd_k (wave = key tile): logits and dA recomputed key-major,
// dK and the key-side sums (Q^T in LDS), then dV from the tile of A kept in
// registers (dO^T in LDS); it adds both sides into dE/dsw and dE/drhat.

template <int NPAD>
__global__ __launch_bounds__(NPAD / 16 * 64, NPAD <= 96 ? 3 : 2) void k_attn_bwd_q(
    const float *__restrict__ qkv, const float *__restrict__ o, const float *__restrict__ dO,
    const float *__restrict__ geom, const int *__restrict__ pair_off,
    const int *__restrict__ nnei, int sel, float shift, float *__restrict__ dqkv,
    float4 *__restrict__ astat, float4 *__restrict__ qside, int nlo) {
  constexpr int NT = NPAD / 16;
  extern __shared__ float4 smem[];
  float4 *kg = smem;                // [NPAD] rhat, sw
  float *XT = (float *)(kg + NPAD);  // [128][NPAD + 4]
  const int i = blockIdx.x;
  const int n = nnei[i];
  if (n <= nlo || n > NPAD) return;  // uniform over the block
  const int base = pair_off[i];
  const int ntile = (n + 15) >> 4;
  const int ld = kQKV * 128;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const float inv_sqrt_d = 0.08838834764831845f;

  stage_gate<NPAD>(geom, base, n, kg);
  stage_t<NPAD>(qkv + 128, ld, base, n, XT);  // K^T
  __syncthreads();

  // ---------------- phase A: wave = query tile
  if (wave < ntile) {
    const int q = wave * 16 + r;
    const bool qok = q < n;
    const float4 gq = kg[q];
    const float wq = qok ? gq.w : 0.f;
    floatx4 lam[NT];
    {
      floatx4 qv[8];
      load_rows(qkv, ld, base, n, q, g, qv);
      qk_tiles<NT>(qkv + 128, ld, base, n, ntile, r, g, qv, lam);
    }
    float mx = -FLT_MAX;
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 16 + 4 * g + v;
        lam[kt][v] *= inv_sqrt_d;
        const float l = k < n ? (lam[kt][v] + shift) * wq * kg[k].w - shift : -INFINITY;
        mx = fmaxf(mx, l);
      }
    }
    const float m = fmaxf(max_groups(mx), -shift);
    float z = 0.f;
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
  #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 16 + 4 * g + v;
        if (k < n) z += expf((lam[kt][v] + shift) * wq * kg[k].w - shift - m);
      }
    }
    z = sum_groups(z) + (float)(sel - n) * expf(-shift - m);
    const float invz = 1.0f / z;

    floatx4 da[NT];
    float dq;
    {
      floatx4 dov[8], ov[8];
      load_rows(dO, 128, base, n, q, g, dov);
      load_rows(o, 128, base, n, q, g, ov);
      dq = 0.f;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        dq += dov[c][0] * ov[c][0] + dov[c][1] * ov[c][1] + dov[c][2] * ov[c][2] +
              dov[c][3] * ov[c][3];
      dq = sum_groups(dq);
      qk_tiles<NT>(qkv + 256, ld, base, n, ntile, r, g, dov, da);  // dA^T tiles
    }
    if (g == 0 && qok) astat[base + q] = make_float4(m, invz, dq, 0.f);

    floatx4 dqacc[8];
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) dqacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
    float dwq = 0.f, drqx = 0.f, drqy = 0.f, drqz = 0.f;
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
        floatx4 ds;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kt * 16 + 4 * g + v;
        const float4 gk = kg[k];
        const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
        const float ww = wq * gk.w;
        const float l = (lam[kt][v] + shift) * ww - shift;
        const float p = (qok && k < n) ? expf(l - m) * invz : 0.f;
        const float h = ww * c;
        const float dH = da[kt][v] * p;
        const float dL = p * (da[kt][v] * h - dq);
        ds[v] = dL * ww * inv_sqrt_d;
        const float X = dL * (lam[kt][v] + shift) + dH * c;
        const float Y = dH * ww;
        dwq += X * gk.w;
        drqx += Y * gk.x;
        drqy += Y * gk.y;
        drqz += Y * gk.z;
      }
      accum_lds<NPAD>(XT, kt, r, g, ds, dqacc);
    }
    dwq = sum_groups(dwq);
    drqx = sum_groups(drqx);
    drqy = sum_groups(drqy);
    drqz = sum_groups(drqz);
    if (g == 0 && qok) qside[base + q] = make_float4(dwq, drqx, drqy, drqz);
    if (qok) {
      float *dp = dqkv + (size_t)(base + q) * ld + 4 * g;
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) *(floatx4 *)(dp + 16 * ft) = dqacc[ft];
    }
  }
}

template <int NPAD>
__global__ __launch_bounds__(NPAD / 16 * 64, NPAD <= 96 ? 3 : 2) void k_attn_bwd_k(
    const float *__restrict__ qkv, const float *__restrict__ dO,
    const float *__restrict__ geom, const int *__restrict__ pair_off,
    const int *__restrict__ nnei, float shift, float *__restrict__ dqkv,
    const float4 *__restrict__ astat, const float4 *__restrict__ qsbuf,
    float *__restrict__ gw, float *__restrict__ gr, int accumulate, int nlo) {
  constexpr int NT = NPAD / 16;
  extern __shared__ float4 smem[];
  float4 *kg = smem;                 // [NPAD] rhat, sw
  float4 *stats = kg + NPAD;         // [NPAD] m, 1/Z, D_q of each query
  float *XT = (float *)(stats + NPAD);  // [128][NPAD + 4]
  const int i = blockIdx.x;
  const int n = nnei[i];
  if (n <= nlo || n > NPAD) return;  // uniform over the block
  const int base = pair_off[i];
  const int ntile = (n + 15) >> 4;
  const int ld = kQKV * 128;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const float inv_sqrt_d = 0.08838834764831845f;
  stage_gate<NPAD>(geom, base, n, kg);
  for (int t = threadIdx.x; t < NPAD; t += blockDim.x)
    stats[t] = t < n ? astat[base + t] : make_float4(0.f, 1.f, 0.f, 0.f);
  stage_t<NPAD>(qkv, ld, base, n, XT);  // Q^T
  __syncthreads();

  // ---------------- phase B1: wave = key tile
  const int kk = wave * 16 + r;
  const bool kok = kk < n;
  floatx4 at[NT];
  float dwk = 0.f, drkx = 0.f, drky = 0.f, drkz = 0.f;
  if (wave < ntile) {
    const float4 gk = kg[kk];
    const float wk = kok ? gk.w : 0.f;
    // logits and dA for this key tile against every query tile, key-major:
    // lane holds key r and queries 4g + v of each query tile
    floatx4 sk[NT], dk[NT];
    {
      floatx4 kreg[8];
      load_rows(qkv + 128, ld, base, n, kk, g, kreg);
      qk_tiles<NT>(qkv, ld, base, n, ntile, r, g, kreg, sk);
    }
    {
      floatx4 vreg[8];
      load_rows(qkv + 256, ld, base, n, kk, g, vreg);
      qk_tiles<NT>(dO, 128, base, n, ntile, r, g, vreg, dk);
    }
    floatx4 dkacc[8];
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) dkacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int qt = 0; qt < NT; ++qt) {
      at[qt] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (qt >= ntile) continue;
      floatx4 ds;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int qq = qt * 16 + 4 * g + v;
        const float4 sq = stats[qq];
        const float4 gq = kg[qq];
        const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
        const float ww = gq.w * wk;
        const float lm = sk[qt][v] * inv_sqrt_d;
        const float l = (lm + shift) * ww - shift;
        const float p = (kok && qq < n) ? expf(l - sq.x) * sq.y : 0.f;
        const float h = ww * c;
        const float dav = dk[qt][v];
        const float dH = dav * p;
        const float dL = p * (dav * h - sq.z);
        at[qt][v] = p * h;
        ds[v] = dL * ww * inv_sqrt_d;
        const float X = dL * (lm + shift) + dH * c;
        const float Y = dH * ww;
        dwk += X * gq.w;
        drkx += Y * gq.x;
        drky += Y * gq.y;
        drkz += Y * gq.z;
      }
      accum_lds<NPAD>(XT, qt, r, g, ds, dkacc);
    }
    if (kok) {
      float *dp = dqkv + (size_t)(base + kk) * ld + 128 + 4 * g;
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) *(floatx4 *)(dp + 16 * ft) = dkacc[ft];
    }
    dwk = sum_groups(dwk);
    drkx = sum_groups(drkx);
    drky = sum_groups(drky);
    drkz = sum_groups(drkz);
  }
  __syncthreads();
  stage_t<NPAD>(dO, 128, base, n, XT);  // dO^T
  __syncthreads();

  // ---------------- phase B2: dV = A^T dO
  if (wave < ntile) {
    floatx4 dvacc[8];
#pragma unroll
    for (int ft = 0; ft < 8; ++ft) dvacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int qt = 0; qt < NT; ++qt)
      if (qt < ntile) accum_lds<NPAD>(XT, qt, r, g, at[qt], dvacc);
    if (kok) {
      float *dp = dqkv + (size_t)(base + kk) * ld + 256 + 4 * g;
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) *(floatx4 *)(dp + 16 * ft) = dvacc[ft];
      if (g == 0) {
        const float4 qs = qsbuf[base + kk];
        const size_t p = (size_t)(base + kk);
        const float tw = qs.x + dwk, tx = qs.y + drkx, ty = qs.z + drky, tz = qs.w + drkz;
        if (accumulate) {
          gw[p] += tw;
          gr[4 * p + 0] += tx;
          gr[4 * p + 1] += ty;
          gr[4 * p + 2] += tz;
        } else {
          gw[p] = tw;
          gr[4 * p + 0] = tx;
          gr[4 * p + 1] = ty;
          gr[4 * p + 2] = tz;
          gr[4 * p + 3] = 0.f;
        }
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
#pragma unroll 4
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
// layer-norm backward of the last attention layer (ln_mode 0), the tanh
// backward of the last embedding layer (ln_mode 1), or dG only (ln_mode 2).
// Sixteen lanes share a pair (lane li holds features li + 16k), so the row
// reductions take four cross-lane steps and four pairs run per wavefront.
__global__ __launch_bounds__(256) void k_desc_bwd(
    const float *__restrict__ geom, const float *__restrict__ G, int ldg,
    const float *__restrict__ T, const float *__restrict__ dD, int ldd,
    const int *__restrict__ pair_off, const int *__restrict__ nnei, int sel, int M, int axis,
    int ln_mode, const float *__restrict__ gamma, const float *__restrict__ xhat,
    const float *__restrict__ rstd, const float *__restrict__ temb, float *__restrict__ dG,
    float *__restrict__ dnext, float *__restrict__ dRt) {
  constexpr int KF = 8;  // features per lane: 16 lanes x 8 = 128 >= ldg
  __shared__ float Ts[4][128];
  __shared__ float dTs[4][128];
  __shared__ float part[16][16][4];
  const int i = blockIdx.x;
  const int n = nnei[i];
  const int base = pair_off[i];
  const int tid = threadIdx.x;
  if (tid < 128) {
    for (int c = 0; c < 4; ++c) Ts[c][tid] = tid < M ? T[(size_t)i * 4 * M + c * M + tid] : 0.f;
  }
  __syncthreads();
  const float *dr = dD + (size_t)i * ldd;
  // second term, spread over all threads: a = tid % 16, rows m' = tid/16 + 16k
  {
    const int aa = tid & 15, pp = tid >> 4;
    float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
    if (aa < axis) {
      for (int mm = pp; mm < M; mm += 16) {
        const float x = dr[mm * axis + aa];
        q0 += x * Ts[0][mm];
        q1 += x * Ts[1][mm];
        q2 += x * Ts[2][mm];
        q3 += x * Ts[3][mm];
      }
    }
    part[pp][aa][0] = q0;
    part[pp][aa][1] = q1;
    part[pp][aa][2] = q2;
    part[pp][aa][3] = q3;
  }
  __syncthreads();
  const float inv = 1.0f / (float)sel;
  if (tid < 128) {
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
    if (tid < M) {
      for (int a = 0; a < axis; ++a) {
        const float x = dr[tid * axis + a];
        d0 += x * Ts[0][a];
        d1 += x * Ts[1][a];
        d2 += x * Ts[2][a];
        d3 += x * Ts[3][a];
      }
      if (tid < axis && tid < 16) {
        for (int pp = 0; pp < 16; ++pp) {
          d0 += part[pp][tid][0];
          d1 += part[pp][tid][1];
          d2 += part[pp][tid][2];
          d3 += part[pp][tid][3];
        }
      }
    }
    dTs[0][tid] = d0 * inv;
    dTs[1][tid] = d1 * inv;
    dTs[2][tid] = d2 * inv;
    dTs[3][tid] = d3 * inv;
  }
  __syncthreads();
  const int grp = tid >> 4, li = tid & 15;
  const float invm = 1.0f / (float)M;
  for (int j = grp; j < n; j += 16) {
    const size_t p = (size_t)(base + j);
    const float *gp = geom + p * kGeom;
    const float s = gp[G_S];
    const float R0 = s, R1 = s * gp[G_RX], R2 = s * gp[G_RY], R3 = s * gp[G_RZ];
    float dg[KF], xh[KF];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int m = li + 16 * k;
      dg[k] = 0.f;
      xh[k] = 0.f;
      if (m < M) {
        const float gm = G[p * ldg + m];
        const float v = R0 * dTs[0][m] + R1 * dTs[1][m] + R2 * dTs[2][m] + R3 * dTs[3][m];
        dg[k] = v;
        a0 += gm * dTs[0][m];
        a1 += gm * dTs[1][m];
        a2 += gm * dTs[2][m];
        a3 += gm * dTs[3][m];
        if (ln_mode == 0) {
          xh[k] = xhat[p * ldg + m];
          const float dx = gamma[m] * v;
          s1 += dx;
          s2 += dx * xh[k];
        }
      }
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
      a3 += __shfl_xor(a3, off);
      s1 += __shfl_xor(s1, off);
      s2 += __shfl_xor(s2, off);
    }
    const float rs = ln_mode == 0 ? rstd[p] : 0.f;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int m = li + 16 * k;
      if (m < ldg) {
        float nx = 0.f;
        if (m < M) {
          if (ln_mode == 0) {
            nx = rs * (gamma[m] * dg[k] - s1 * invm - xh[k] * s2 * invm);
          } else if (ln_mode == 1) {
            const float t = temb[p * ldg + m];
            nx = dg[k] * (1.0f - t * t);
          }
        }
        dG[p * ldg + m] = dg[k];
        if (ln_mode != 2) dnext[p * ldg + m] = nx;
      }
    }
    if (li == 0) *(float4 *)(dRt + 4 * p) = make_float4(a0, a1, a2, a3);
  }
}

// Centres are grouped by neighbour count into classes of 32, 64, 96 and 128
// slots; each class runs a kernel sized for it (blocks of the other classes
// exit at once), so the common case does not pay for the largest LDS size.
template <int NPAD>
size_t fwd_lds() {
  return sizeof(float4) * NPAD + sizeof(float) * 128 * (NPAD + 4);
}
template <int NPAD>
size_t bwdq_lds() {
  return sizeof(float4) * NPAD + sizeof(float) * 128 * (NPAD + 4);
}
template <int NPAD>
size_t bwdk_lds() {
  return sizeof(float4) * 2 * NPAD + sizeof(float) * 128 * (NPAD + 4);
}

template <int NPAD>
void fwd_one(const float *qkv, const float *geom, const int *pair_off, const int *nnei, int nloc,
             int sel, float shift, float *out, int nlo, hipStream_t s) {
  hipLaunchKernelGGL(k_attn_fwd<NPAD>, dim3(nloc), dim3(NPAD / 16 * 64), fwd_lds<NPAD>(), s, qkv,
                     geom, pair_off, nnei, sel, shift, out, nlo);
}
template <int NPAD>
void bwdq_one(const float *qkv, const float *o, const float *dO, const float *geom,
              const int *pair_off, const int *nnei, int nloc, int sel, float shift, float *dqkv,
              float4 *astat, float4 *qside, int nlo, hipStream_t s) {
  hipLaunchKernelGGL(k_attn_bwd_q<NPAD>, dim3(nloc), dim3(NPAD / 16 * 64), bwdq_lds<NPAD>(), s,
                     qkv, o, dO, geom, pair_off, nnei, sel, shift, dqkv, astat, qside, nlo);
}
template <int NPAD>
void bwdk_one(const float *qkv, const float *dO, const float *geom, const int *pair_off,
              const int *nnei, int nloc, float shift, float *dqkv, const float4 *astat,
              const float4 *qside, float *gw, float *gr, int accumulate, int nlo, hipStream_t s) {
  hipLaunchKernelGGL(k_attn_bwd_k<NPAD>, dim3(nloc), dim3(NPAD / 16 * 64), bwdk_lds<NPAD>(), s,
                     qkv, dO, geom, pair_off, nnei, shift, dqkv, astat, qside, gw, gr, accumulate,
                     nlo);
}

}  // namespace

int attn_class_count(int sel) { return sel <= 32 ? 1 : sel <= 64 ? 2 : sel <= 96 ? 3 : 4; }
int attn_class_npad(int cls) { return 32 * (cls + 1); }

void launch_attn_fwd_class(int cls, const float *qkv, const float *geom, const int *pair_off,
                           const int *nnei, int nloc, int sel, float shift, float *out,
                           hipStream_t s) {
  if (nloc <= 0) return;
  switch (cls) {
    case 0: fwd_one<32>(qkv, geom, pair_off, nnei, nloc, sel, shift, out, 0, s); break;
    case 1: fwd_one<64>(qkv, geom, pair_off, nnei, nloc, sel, shift, out, 32, s); break;
    case 2: fwd_one<96>(qkv, geom, pair_off, nnei, nloc, sel, shift, out, 64, s); break;
    default: fwd_one<128>(qkv, geom, pair_off, nnei, nloc, sel, shift, out, 96, s); break;
  }
}

void launch_attn_bwd_q_class(int cls, const float *qkv, const float *o, const float *dO,
                             const float *geom, const int *pair_off, const int *nnei, int nloc,
                             int sel, float shift, float *dqkv, float *astat, float *qside,
                             hipStream_t s) {
  if (nloc <= 0) return;
  float4 *a4 = (float4 *)astat, *q4 = (float4 *)qside;
  switch (cls) {
    case 0: bwdq_one<32>(qkv, o, dO, geom, pair_off, nnei, nloc, sel, shift, dqkv, a4, q4, 0, s); break;
    case 1: bwdq_one<64>(qkv, o, dO, geom, pair_off, nnei, nloc, sel, shift, dqkv, a4, q4, 32, s); break;
    case 2: bwdq_one<96>(qkv, o, dO, geom, pair_off, nnei, nloc, sel, shift, dqkv, a4, q4, 64, s); break;
    default: bwdq_one<128>(qkv, o, dO, geom, pair_off, nnei, nloc, sel, shift, dqkv, a4, q4, 96, s); break;
  }
}

void launch_attn_bwd_k_class(int cls, const float *qkv, const float *dO, const float *geom,
                             const int *pair_off, const int *nnei, int nloc, float shift,
                             float *dqkv, const float *astat, const float *qside, float *gw,
                             float *gr, int accumulate, hipStream_t s) {
  if (nloc <= 0) return;
  const float4 *a4 = (const float4 *)astat, *q4 = (const float4 *)qside;
  switch (cls) {
    case 0: bwdk_one<32>(qkv, dO, geom, pair_off, nnei, nloc, shift, dqkv, a4, q4, gw, gr, accumulate, 0, s); break;
    case 1: bwdk_one<64>(qkv, dO, geom, pair_off, nnei, nloc, shift, dqkv, a4, q4, gw, gr, accumulate, 32, s); break;
    case 2: bwdk_one<96>(qkv, dO, geom, pair_off, nnei, nloc, shift, dqkv, a4, q4, gw, gr, accumulate, 64, s); break;
    default: bwdk_one<128>(qkv, dO, geom, pair_off, nnei, nloc, shift, dqkv, a4, q4, gw, gr, accumulate, 96, s); break;
  }
}

hipError_t set_attn_bwd_lds_limit() {
  hipError_t e = hipFuncSetAttribute((const void *)k_attn_bwd_q<128>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bwdq_lds<128>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_attn_bwd_k<128>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwdk_lds<128>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_attn_fwd<128>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_lds<128>());
  return e;
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
