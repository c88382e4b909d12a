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
#include "ln_res.h"

namespace dpa1 {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kMaxTiles = 8;     // 128 neighbours
constexpr int kQKV = 3;          // q, k, v blocks in one row of the projection output

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 precision mode (template flag BF): gfx950's v_mfma_f32_16x16x32_bf16
// contracts two 16-deep chunks (two feature chunks, or two 16-neighbour
// tiles) at once.  Each lane's eight operand slots hold its four
// consecutive k values of the first chunk, then those of the second, on
// both operands alike (the values the FP32 path feeds to four 16x16x4 steps
// per chunk), which equals two 16x16x16 steps.  Operands are rounded to BF16
// in registers, accumulation is FP32.  Every class has an even number of
// tiles, so tiles always pair.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x4 to_bf16(const floatx4 &v) {
  return __builtin_convertvector(v, bf16x4);
}
__device__ __forceinline__ bf16x8 to_bf16x8(const floatx4 &lo, const floatx4 &hi) {
  return __builtin_shufflevector(to_bf16(lo), to_bf16(hi), 0, 1, 2, 3, 4, 5, 6, 7);
}
__device__ __forceinline__ floatx4 mfma_bf16x2(const bf16x8 &a, const bf16x8 &b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// exp x = 2^(x log2 e) on the hardware v_exp_f32: two operations instead of
// the library expf's range reduction.  Its arguments here are logits minus
// their row maximum (<= 0); the relative error, about |x| ulps, is below the
// FP32 rounding of what follows.  The forward and both adjoint kernels use
// it alike, so the adjoint recomputes the forward's probabilities exactly.
__device__ __forceinline__ float exp_hw(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
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

// Pair tensors (QKV, the attention output o, dO, dQKV) are stored FP32, or
// BF16 in BF16 mode (SB), where they are only ever BF16 matrix-core operands
// (the one elementwise use, D_q = dO . o, then sees the rounded values).
// Offsets are in elements of the storage type.
template <bool SB>
__device__ __forceinline__ const float *pt_at(const float *base, size_t e) {
  if constexpr (SB) return (const float *)((const __bf16 *)base + e);
  else return base + e;
}
template <bool SB>
__device__ __forceinline__ float *pt_at(float *base, size_t e) {
  if constexpr (SB) return (float *)((__bf16 *)base + e);
  else return base + e;
}
template <bool SB>
__device__ __forceinline__ floatx4 ldp4(const float *p, int e) {
  if constexpr (SB)
    return __builtin_convertvector(*(const bf16x4 *)((const __bf16 *)p + e), floatx4);
  else
    return *(const floatx4 *)(p + e);
}
template <bool SB>
__device__ __forceinline__ void stp4(float *p, int e, const floatx4 &v) {
  if constexpr (SB)
    *(bf16x4 *)((__bf16 *)p + e) = __builtin_convertvector(v, bf16x4);
  else
    *(floatx4 *)(p + e) = v;
}

// Load one 16x128 row tile (columns col..col+127) as the MFMA B operand:
// lane holds row r, features 16c + 4g + {0..3}.  Rows past n read row 0 of
// the centre (finite values; every use of such a row is masked), so no load
// waits on a select.
template <bool SB>
__device__ __forceinline__ void load_rows(const float *__restrict__ rows, int col, int ld,
                                          int base, int n, int row, int g, floatx4 (&v)[8]) {
  const float *rb = pt_at<SB>(rows, (size_t)base * ld + col);
  const int off = (row < n ? row : 0) * ld + 4 * g;
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = ldp4<SB>(rb, off + 16 * c);
}

// Row stride of the row-major LDS tiles: 128 features + 4 (with it, eight
// consecutive lanes reading 16 bytes each from eight consecutive rows touch
// 32 distinct banks).
constexpr int kLDR = 132;

// Stage rows [base, base + n) x 128 features of src (row stride ld) into LDS
// row-major, X[row][kLDR]; rows n..NPAD-1 are zero.  Products whose A operand
// runs along the features (Q K^T, dO V^T) read it with one 16-byte LDS load
// per lane per four MFMA steps.
// The loads and the LDS writes are separate steps so that a kernel issues
// every global load of a phase before it waits for any (a load whose value is
// consumed at once, or a branch that overwrites it, serialises the latencies).
// Rows past n read row 0 and are written as zeros (a select at the write).
template <int NPAD, bool SB>
__device__ __forceinline__ void stage_rows_load(const float *__restrict__ src, int col, int ld,
                                                int base, int n, int tid, float4 (&v)[8]) {
  constexpr int THREADS = NPAD / 16 * 64;
  static_assert(NPAD * 32 / THREADS == 8, "eight float4 per thread");
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const int idx = tid + it * THREADS;
    const int row = idx >> 5, c4 = idx & 31;
    const int rr = row < n ? row : 0;
    const floatx4 x = ldp4<SB>(pt_at<SB>(src, (size_t)(base + rr) * ld + col + 4 * c4), 0);
    v[it] = make_float4(x[0], x[1], x[2], x[3]);
  }
}
template <int NPAD>
__device__ __forceinline__ void stage_rows_store(float *X, int tid, int n, const float4 (&v)[8]) {
  constexpr int THREADS = NPAD / 16 * 64;
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const int idx = tid + it * THREADS;
    const int row = idx >> 5, c4 = idx & 31;
    const bool ok = row < n;
    *(float4 *)(X + row * kLDR + 4 * c4) =
        make_float4(ok ? v[it].x : 0.f, ok ? v[it].y : 0.f, ok ? v[it].z : 0.f, ok ? v[it].w : 0.f);
  }
}

// Stage rows [base, base + n) x 128 features of src into LDS transposed,
// XT[f][k] with row stride NPAD + 4; rows n..NPAD-1 are zero.  Products that
// contract over neighbours read it with one 16-byte LDS load per lane per
// four MFMA steps.  Wave w stages rows 16w..16w+15; in each step lane l takes
// row 16w + l%16 and feature quad 4 it + l/16, so the four scalar LDS writes
// of one float4 hit 64 distinct banks.
// The load half and the LDS half are separate so that a kernel can issue the
// loads one phase early (while the previous phase computes) and write LDS
// after the barrier that frees the buffer.
template <int NPAD, bool SB>
__device__ __forceinline__ void stage_t_load(const float *__restrict__ src, int col, int ld,
                                             int base, int n, int tid, float4 (&v)[8]) {
  const int row = (tid >> 6) * 16 + (tid & 15);
  const int cq = (tid >> 4) & 3;
  const int rr = row < n ? row : 0;
  const float *sp = pt_at<SB>(src, (size_t)(base + rr) * ld + col + 4 * cq);
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const floatx4 x = ldp4<SB>(sp, 16 * it);
    v[it] = make_float4(x[0], x[1], x[2], x[3]);
  }
}
// rows past n (loaded from row 0) are written as zeros
template <int NPAD>
__device__ __forceinline__ void stage_t_store(float *XT, int tid, int n, const float4 (&v)[8]) {
  constexpr int LDT = NPAD + 4;
  const int row = (tid >> 6) * 16 + (tid & 15);
  const int cq = (tid >> 4) & 3;
  const bool ok = row < n;
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    float *d = XT + (16 * it + 4 * cq) * LDT + row;
    d[0] = ok ? v[it].x : 0.f;
    d[LDT] = ok ? v[it].y : 0.f;
    d[2 * LDT] = ok ? v[it].z : 0.f;
    d[3 * LDT] = ok ? v[it].w : 0.f;
  }
}

// Gate record of neighbour t = tid (rhat, sw; zeros past n), for kg[NPAD]:
// one unconditional load per thread (threads past NPAD read slot 0), written
// by gate_store.  lo is the FP32 remainder of the switch value (sw - hi in
// FP64), so that hi + lo carries sw to the logits with FP64 accuracy.
__device__ __forceinline__ float4 gate_load(const float *__restrict__ geom, int base, int n,
                                            int tid, float &lo) {
  const int t = tid < n ? tid : 0;
  const float4 *gp = (const float4 *)(geom + (size_t)(base + t) * kGeom);
  const float4 a = gp[0], b = gp[1];  // s, rx, ry, rz | sw, r, dsw, sw remainder
  lo = b.w;
  return make_float4(a.y, a.z, a.w, b.x);
}
// kw[NPAD]: the switch value of each neighbour in FP64 (zero past n).
template <int NPAD>
__device__ __forceinline__ void gate_store(float4 *kg, double *kw, int tid, int n,
                                           const float4 &v, float lo) {
  const bool ok = tid < n;
  if (tid < NPAD) {
    kg[tid] = make_float4(ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f);
    kw[tid] = ok ? (double)v.w + (double)lo : 0.0;
  }
}

// Scaled logit L = (lam + S) w_q w_k - S of the FP32 path, with the switch
// values and the shift in FP64 and one rounding at the end.  The logit's
// sensitivity to each switch value is lam + S (about S = 20), so with FP32
// switch values and FP32 arithmetic here the logit carries an absolute error
// of a few 1e-6; at the rare centres where a pair of opposite neighbours
// attend strongly to each other the forces amplify that by ~1e4 (measured on
// the oracle's formula evaluated in FP32).  The products and every other
// elementwise step stay FP32; the BF16 mode keeps FP32 logits.
__device__ __forceinline__ float logit64(float lam, double wq, double wk, float shift) {
  const double s = (double)shift;
  return (float)fma((double)lam + s, wq * wk, -s);
}

// acc[ft] += XT^T-tile x bt : contraction over the 16 rows of tile 'tile',
// XT in LDS (feature-major), bt a 16x16 B operand held in registers.
// Output lane layout: own row r, features 16 ft + 4 g + v.
template <int NPAD>
__device__ __forceinline__ void accum_lds(const float *XT, int tile, int r, int g,
                                          const floatx4 &bt, floatx4 (&acc)[8]) {
  constexpr int LDT = NPAD + 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {  // two halves of the features: 16 operand registers
    floatx4 x[4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
      x[f] = *(const floatx4 *)(XT + ((4 * h + f) * 16 + r) * LDT + tile * 16 + 4 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[4 * h + f] = mfma4(x[f][t], bt[t], acc[4 * h + f]);
  }
}
// BF16: tiles 'tile' and 'tile' + 1 in one 16x16x32 step, B operands bt0, bt1.
template <int NPAD>
__device__ __forceinline__ void accum_lds2(const float *XT, int tile, int r, int g,
                                           const floatx4 &bt0, const floatx4 &bt1,
                                           floatx4 (&acc)[8]) {
  constexpr int LDT = NPAD + 4;
  const bf16x8 btb = to_bf16x8(bt0, bt1);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    floatx4 x0[4], x1[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const float *xp = XT + ((4 * h + f) * 16 + r) * LDT + tile * 16 + 4 * g;
      x0[f] = *(const floatx4 *)xp;
      x1[f] = *(const floatx4 *)(xp + 16);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f)
      acc[4 * h + f] = mfma_bf16x2(to_bf16x8(x0[f], x1[f]), btb, acc[4 * h + f]);
  }
}

// The same contraction with the rows in row-major LDS (X[row][kLDR]): the A
// operand is read with scalar LDS loads, four rows per lane group.
__device__ __forceinline__ void accum_rows(const float *X, int tile, int r, int g,
                                           const floatx4 &bt, floatx4 (&acc)[8]) {
  const float *xb = X + (tile * 16 + 4 * g) * kLDR + r;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    floatx4 x[4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int t = 0; t < 4; ++t) x[f][t] = xb[t * kLDR + (4 * h + f) * 16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[4 * h + f] = mfma4(x[f][t], bt[t], acc[4 * h + f]);
  }
}
// BF16: row tiles 'tile' and 'tile' + 1 in one 16x16x32 step.
__device__ __forceinline__ void accum_rows2(const float *X, int tile, int r, int g,
                                            const floatx4 &bt0, const floatx4 &bt1,
                                            floatx4 (&acc)[8]) {
  const float *xb = X + (tile * 16 + 4 * g) * kLDR + r;
  const bf16x8 btb = to_bf16x8(bt0, bt1);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    floatx4 x0[4], x1[4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        x0[f][t] = xb[t * kLDR + (4 * h + f) * 16];
        x1[f][t] = xb[(16 + t) * kLDR + (4 * h + f) * 16];
      }
#pragma unroll
    for (int f = 0; f < 4; ++f)
      acc[4 * h + f] = mfma_bf16x2(to_bf16x8(x0[f], x1[f]), btb, acc[4 * h + f]);
  }
}

// st[kt] (lane: own row r, tile rows 4g + v) = X-rows of tile kt times the
// wave's own 16 rows b, contracted over the 128 features; X row-major in LDS.
template <int NT, bool BF>
__device__ __forceinline__ void qk_lds(const float *X, int r, int g, const floatx4 (&b)[8],
                                       floatx4 (&st)[NT]) {
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) st[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
  const float *xb = X + r * kLDR + 4 * g;
  // one feature chunk at a time (LDS latency is covered by the other
  // wavefronts on the SIMD); the fence keeps the compiler from hoisting the
  // loads of later chunks, which would hold many more registers
  if constexpr (BF) {
    // feature chunks 2h and 2h + 1 in one 16x16x32 step
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      floatx4 a0[NT], a1[NT];
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) {
        a0[kt] = *(const floatx4 *)(xb + kt * 16 * kLDR + 32 * h);
        a1[kt] = *(const floatx4 *)(xb + kt * 16 * kLDR + 32 * h + 16);
      }
      __builtin_amdgcn_sched_barrier(0);
      const bf16x8 bb = to_bf16x8(b[2 * h], b[2 * h + 1]);
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) st[kt] = mfma_bf16x2(to_bf16x8(a0[kt], a1[kt]), bb, st[kt]);
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    floatx4 a[NT];
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) a[kt] = *(const floatx4 *)(xb + kt * 16 * kLDR + 16 * c);
    __builtin_amdgcn_sched_barrier(0);
    {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) st[kt] = mfma4(a[kt][t], b[c][t], st[kt]);
    }
  }
}

// The thread index, opaque to the optimiser.  Taken afresh in every
// iteration of the per-centre loops so that per-lane addresses are
// recomputed there instead of being hoisted out of the loop and held in
// registers for its whole duration (which made the large classes spill).
__device__ __forceinline__ int fresh_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Floats of the staging buffer: NPAD rows x kLDR or 128 features x (NPAD + 4).
template <int NPAD>
constexpr int stage_floats() {
  return NPAD * kLDR > 128 * (NPAD + 4) ? NPAD * kLDR : 128 * (NPAD + 4);
}

// --------------------------------------------------------------------- forward
//
// Centres are processed by a persistent grid: block b takes the centres
// b, b + gridDim.x, ... of its class list (every centre of a class costs the
// same padded work, so the static split is balanced).  One wavefront per
// 16-query tile.  K is staged row-major in LDS for Q K^T, then V transposed
// for A V; global memory is touched only by the staging steps, the wave's
// own query rows and the outputs.  The scaled dot products lam = q.k/sqrt(d)
// (row stride kLamLd, all NPAD key columns of every query row) and the
// softmax statistics (m, 1/Z) of every query are stored for the adjoint,
// which then does not recompute Q K^T.  The FP32 forward issues the next
// centre's staging loads during its last phase, into registers the current
// centre no longer needs, so that the HBM latency of a centre's operands
// overlaps the previous centre's products (two workgroups per compute unit
// leave the registers for it).

constexpr int kLamLd = kAttnLamLd;
constexpr int kOpCols = kAttnOpCols;   // output columns of the fused projection
constexpr int kOpTiles = kOpCols / 16;

// OP: the output projection and its layer norm are applied here
// (W_O^T, 7 column tiles, staged in LDS once per workgroup; the epilogue is
// the one the projection GEMM uses), so the attention output o goes to
// memory only where the two-kernel adjoint of the 128 class reads it.
template <int NPAD, bool BF, bool OP>
__global__ __launch_bounds__(NPAD / 16 * 64, BF && !OP ? (NPAD <= 64 ? 4 : (NPAD <= 96 ? 3 : 2)) : 2) void k_attn_fwd(
    const float *__restrict__ qkv, const float *__restrict__ geom,
    const int *__restrict__ pair_off, const int *__restrict__ nnei,
    const int *__restrict__ clist, const int *__restrict__ ccount, int sel, float shift,
    float *__restrict__ out, float *__restrict__ lam, float2 *__restrict__ fstat,
    AttnOut op) {
  constexpr int NT = NPAD / 16;
  constexpr bool STORE_O = !OP || NPAD > 96;
  extern __shared__ float4 smem[];
  float4 *kg = smem;
  double *kw = (double *)(smem + NPAD);  // [NPAD] switch values in FP64
  float *buf = (float *)(kw + NPAD);     // K rows, then V^T
  float *wo = buf + stage_floats<NPAD>();  // OP: W_O^T [kOpCols][kLDR]
  float *cso = wo + kOpCols * kLDR;        // OP: bias, gamma, beta [3][kOpCols]
  const int ld = kQKV * 128;
  const float inv_sqrt_d = 0.08838834764831845f;  // 1/sqrt(128)
  const int cnt = *ccount;
  if constexpr (OP) {
    for (int idx = threadIdx.x; idx < kOpCols * 32; idx += blockDim.x) {
      const int row = idx >> 5, c4 = idx & 31;
      *(float4 *)(wo + row * kLDR + 4 * c4) = *(const float4 *)(op.Wt_o + row * 128 + 4 * c4);
    }
    for (int idx = threadIdx.x; idx < 3 * kOpCols; idx += blockDim.x) {
      const int k = idx / kOpCols, n = idx % kOpCols;
      cso[idx] = (k == 0 ? op.bias : (k == 1 ? op.gamma : op.beta))[n];
    }
  }
  // FP32: the staging loads of a centre are issued during the A V phase of the
  // previous one (BF16 holds more registers per tile and loads per centre)
  constexpr bool PREF = !BF;
  float4 sv[8];
  floatx4 qv[8];
  float4 gv;
  float gl = 0.f;
  int n_nx = 0, base_nx = 0;
  if (PREF && (int)blockIdx.x < cnt) {
    const int tid = fresh_tid();
    const int i0 = clist[blockIdx.x];
    n_nx = nnei[i0];
    base_nx = pair_off[i0];
    stage_rows_load<NPAD, BF>(qkv, 128, ld, base_nx, n_nx, tid, sv);  // K
    gv = gate_load(geom, base_nx, n_nx, tid, gl);
    load_rows<BF>(qkv, 0, ld, base_nx, n_nx, (tid >> 6) * 16 + (tid & 15), (tid & 63) >> 4, qv);
  }
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int tid = fresh_tid();
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    if constexpr (!PREF) {
      const int i = clist[it];
      n_nx = nnei[i];
      base_nx = pair_off[i];
      stage_rows_load<NPAD, BF>(qkv, 128, ld, base_nx, n_nx, tid, sv);  // K
      gv = gate_load(geom, base_nx, n_nx, tid, gl);
      load_rows<BF>(qkv, 0, ld, base_nx, n_nx, wave * 16 + r, g, qv);
    }
    const int n = n_nx;
    const int base = base_nx;
    const int ntile = (n + 15) >> 4;
    const int q = wave * 16 + r;
    const bool qok = q < n;
    stage_rows_store<NPAD>(buf, tid, n, sv);
    gate_store<NPAD>(kg, kw, tid, n, gv, gl);
    __syncthreads();
    float4 vpre[8];  // V, read while Q K^T and the softmax run
    stage_t_load<NPAD, BF>(qkv, 256, ld, base, n, tid, vpre);

    floatx4 st[NT];
    float invz = 0.f;
    if (wave < ntile) {
      qk_lds<NT, BF>(buf, r, g, qv, st);
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) st[kt] *= inv_sqrt_d;
      if (qok) {
        float *lp = lam + (size_t)(base + q) * kLamLd + 4 * g;
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) *(floatx4 *)(lp + 16 * kt) = st[kt];
      }
      const float wq = qok ? kg[q].w : 0.f;
      const double wqd = qok ? kw[q] : 0.0;
      float mx = -FLT_MAX;
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = kt * 16 + 4 * g + v;
          float l = BF ? (st[kt][v] + shift) * wq * kg[k].w - shift
                       : logit64(st[kt][v], wqd, kw[k], shift);
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
          const float e = exp_hw(st[kt][v] - m);
          st[kt][v] = e;
          z += e;
        }
      }
      z = sum_groups(z) + (float)(sel - n) * exp_hw(-shift - m);
      invz = 1.0f / z;
      if (g == 0 && qok) fstat[base + q] = make_float2(m, invz);
    }
    __syncthreads();
    stage_t_store<NPAD>(buf, tid, n, vpre);  // V^T
    __syncthreads();
    if constexpr (PREF) {
      const int itn = it + (int)gridDim.x;
      if (itn < cnt) {
        const int inx = clist[itn];
        n_nx = nnei[inx];
        base_nx = pair_off[inx];
        stage_rows_load<NPAD, BF>(qkv, 128, ld, base_nx, n_nx, tid, sv);
        gv = gate_load(geom, base_nx, n_nx, tid, gl);
        load_rows<BF>(qkv, 0, ld, base_nx, n_nx, q, g, qv);
      }
    }

    if (wave < ntile) {
      const float4 gq = kg[q];
      const float wq = qok ? gq.w : 0.f;
      floatx4 oacc[8];
      floatx4 atp;  // BF16: probabilities of the even tile of a pair
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
        if constexpr (BF) {  // tiles taken in pairs
          if (kt % 2 == 0) atp = at;
          else accum_lds2<NPAD>(buf, kt - 1, r, g, atp, at, oacc);
        } else {
          accum_lds<NPAD>(buf, kt, r, g, at, oacc);
        }
      }
      if (STORE_O && qok) {
        float *opp = pt_at<BF>(out, (size_t)(base + q) * 128 + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(opp, 16 * ft, oacc[ft]);
      }
      if constexpr (OP) {
        // y = o W_O in the projection GEMM's order (feature chunk, step,
        // column tile), then G_out = G_in + gamma LN(y + b) + beta
        const size_t rb = (size_t)(base + (qok ? q : 0)) * kOpCols;
        floatx4 gi[kOpTiles];
#pragma unroll
        for (int nt = 0; nt < kOpTiles; ++nt) gi[nt] = *(const floatx4 *)(op.gin + rb + 16 * nt + 4 * g);
        floatx4 y[kOpTiles];
#pragma unroll
        for (int nt = 0; nt < kOpTiles; ++nt) y[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        const float *wl = wo + r * kLDR + 4 * g;
        if constexpr (BF) {
          // feature chunks 2h and 2h + 1 in one 16x16x32 step
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const bf16x8 ob = to_bf16x8(oacc[2 * h], oacc[2 * h + 1]);
            bf16x8 w[kOpTiles];
#pragma unroll
            for (int nt = 0; nt < kOpTiles; ++nt)
              w[nt] = to_bf16x8(*(const floatx4 *)(wl + nt * 16 * kLDR + 32 * h),
                                *(const floatx4 *)(wl + nt * 16 * kLDR + 32 * h + 16));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int nt = 0; nt < kOpTiles; ++nt) y[nt] = mfma_bf16x2(w[nt], ob, y[nt]);
          }
        } else {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            floatx4 w[kOpTiles];
#pragma unroll
            for (int nt = 0; nt < kOpTiles; ++nt)
              w[nt] = *(const floatx4 *)(wl + nt * 16 * kLDR + 16 * c);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int nt = 0; nt < kOpTiles; ++nt) y[nt] = mfma4(w[nt][t], oacc[c][t], y[nt]);
          }
        }
        lnres::apply_tile<kOpTiles>(y, gi, g, kOpTiles, op.Nreal, op.eps, cso, kOpCols, qok,
                                    base + q, rb, op.gout, op.xhat, op.rstd);
      }
    }
    __syncthreads();  // LDS is restaged for the next centre
  }
}

// -------------------------------------------------------------------- backward
//
// Given dO, with H = w_q w_k c_qk (c = rhat_q . rhat_k):
//   dA = dO V^T ; dV = A^T dO ; dP = dA H ; dH = dA P
//   D_q = sum_k P dP = dO_q . o_q ; dL = P (dP - D_q)
//   dS = dL w_q w_k / sqrt(d) ; dQ = dS K ; dK = dS^T Q
//   X = dL (lam + S) + dH c  -> dw_q += sum_k X w_k, dw_k += sum_q X w_q
//   Y = dH w_q w_k           -> drhat_q += sum_k Y rhat_k, drhat_k += sum_q Y rhat_q
// Two kernels per class, both reading lam and (m, 1/Z) stored by the forward.
// k_attn_bwd_q (wave = query tile): dA^T from V staged row-major, then dS,
// dQ (K^T staged) and the query-side sums; it writes dA in the layout of lam
// (row = query, n columns), (m, 1/Z, D_q) and the query-side sums per pair.
// k_attn_bwd_k (wave = key tile): reads dA key-major the way it reads lam
// (one column of the centre's rows per lane) instead of forming it a second
// time with a matrix product, forms dV from dO staged row-major, then dK
// (Q^T staged) and the key-side sums; it adds both sides into dE/dsw and
// dE/drhat.

template <int NPAD, bool BF>
__global__ __launch_bounds__(NPAD / 16 * 64, NPAD <= 96 ? 3 : 2) void k_attn_bwd_q(
    const float *__restrict__ qkv, const float *__restrict__ o, const float *__restrict__ dO,
    const float *__restrict__ geom, const int *__restrict__ pair_off,
    const int *__restrict__ nnei, const int *__restrict__ clist, const int *__restrict__ ccount,
    int sel, float shift, const float *__restrict__ lam, const float2 *__restrict__ fstat,
    float *__restrict__ dqkv, float4 *__restrict__ astat, float4 *__restrict__ qside,
    float *__restrict__ dA) {
  constexpr int NT = NPAD / 16;
  extern __shared__ float4 smem[];
  float4 *kg = smem;                     // [NPAD] rhat, sw
  double *kw = (double *)(kg + NPAD);    // [NPAD] switch values in FP64
  float *buf = (float *)(kw + NPAD);     // V rows, then K^T
  const int ld = kQKV * 128;
  const float inv_sqrt_d = 0.08838834764831845f;
  const int cnt = *ccount;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int tid = fresh_tid();
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    const int i = clist[it];
    const int n = nnei[i];
    const int base = pair_off[i];
    const int ntile = (n + 15) >> 4;
    const int q = wave * 16 + r;
    const bool qok = q < n;
    float4 sv[8];
    stage_rows_load<NPAD, BF>(qkv, 256, ld, base, n, tid, sv);  // V
    float gl;
    const float4 gv = gate_load(geom, base, n, tid, gl);
    floatx4 dov[8], ov[8];
    load_rows<BF>(dO, 0, 128, base, n, q, g, dov);
    load_rows<BF>(o, 0, 128, base, n, q, g, ov);
    stage_rows_store<NPAD>(buf, tid, n, sv);
    gate_store<NPAD>(kg, kw, tid, n, gv, gl);
    __syncthreads();
    float dq = 0.f;
    if (wave < ntile) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        dq += dov[c][0] * ov[c][0] + dov[c][1] * ov[c][1] + dov[c][2] * ov[c][2] +
              dov[c][3] * ov[c][3];
      dq = sum_groups(dq);
    }
    float4 kpre[8];  // K, read while dA^T is formed
    stage_t_load<NPAD, BF>(qkv, 128, ld, base, n, tid, kpre);

    floatx4 da[NT];
    if (wave < ntile) {
      qk_lds<NT, BF>(buf, r, g, dov, da);  // dA^T tiles: lane (query r, keys 4g + v)
      if (qok) {  // dA row of this query, for the key-tile kernel
        float *dp = dA + (size_t)(base + q) * kLamLd + 4 * g;
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) *(floatx4 *)(dp + 16 * kt) = da[kt];
      }
    }
    __syncthreads();
    stage_t_store<NPAD>(buf, tid, n, kpre);  // K^T
    __syncthreads();

    if (wave < ntile) {
      const int qr = qok ? q : 0;
      const float4 gq = kg[q];
      const float wq = qok ? gq.w : 0.f;
      const double wqd = qok ? kw[q] : 0.0;
      const float2 fs = fstat[base + qr];
      const float m = fs.x, invz = fs.y;
      if (g == 0 && qok) astat[base + q] = make_float4(m, invz, dq, 0.f);
      // lam of this query row, read one key tile ahead of its use
      const float *lp = lam + (size_t)(base + qr) * kLamLd + 4 * g;
      floatx4 dqacc[8];
      floatx4 dsp;  // BF16: dS of the even tile of a pair
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) dqacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
      float dwq = 0.f, drqx = 0.f, drqy = 0.f, drqz = 0.f;
      floatx4 lcur = *(const floatx4 *)lp, lnxt;
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) {
        if (kt + 1 < NT) lnxt = *(const floatx4 *)(lp + 16 * (kt + 1));
        floatx4 ds;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = kt * 16 + 4 * g + v;
          const bool ok = qok && k < n;
          const float4 gk = kg[k];
          const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
          const float ww = wq * gk.w;
          const float lm = ok ? lcur[v] : 0.f;
          const float l = BF ? (lm + shift) * ww - shift : logit64(lm, wqd, kw[k], shift);
          const float p = ok ? exp_hw(l - m) * invz : 0.f;
          const float h = ww * c;
          const float dH = da[kt][v] * p;
          const float dL = p * (da[kt][v] * h - dq);
          ds[v] = dL * ww * inv_sqrt_d;
          const float X = dL * (lm + shift) + dH * c;
          const float Y = dH * ww;
          dwq += X * gk.w;
          drqx += Y * gk.x;
          drqy += Y * gk.y;
          drqz += Y * gk.z;
        }
        if constexpr (BF) {  // tiles taken in pairs
          if (kt % 2 == 0) dsp = ds;
          else accum_lds2<NPAD>(buf, kt - 1, r, g, dsp, ds, dqacc);
        } else {
          accum_lds<NPAD>(buf, kt, r, g, ds, dqacc);
        }
        lcur = lnxt;
      }
      dwq = sum_groups(dwq);
      drqx = sum_groups(drqx);
      drqy = sum_groups(drqy);
      drqz = sum_groups(drqz);
      if (g == 0 && qok) qside[base + q] = make_float4(dwq, drqx, drqy, drqz);
      if (qok) {
        float *dp = pt_at<BF>(dqkv, (size_t)(base + q) * ld + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(dp, 16 * ft, dqacc[ft]);
      }
    }
    __syncthreads();  // LDS is restaged for the next centre
  }
}

template <int NPAD, bool BF>
__global__ __launch_bounds__(NPAD / 16 * 64, BF ? (NPAD <= 96 ? 3 : 2) : 2) void k_attn_bwd_k(
    const float *__restrict__ qkv, const float *__restrict__ dO,
    const float *__restrict__ geom, const int *__restrict__ pair_off,
    const int *__restrict__ nnei, const int *__restrict__ clist, const int *__restrict__ ccount,
    float shift, const float *__restrict__ lam, const float *__restrict__ dA,
    float *__restrict__ dqkv, const float4 *__restrict__ astat,
    const float4 *__restrict__ qsbuf, float *__restrict__ gw, float *__restrict__ gr,
    int accumulate) {
  constexpr int NT = NPAD / 16;
  extern __shared__ float4 smem[];
  float4 *kg = smem;                     // [NPAD] rhat, sw
  float4 *stats = kg + NPAD;             // [NPAD] m, 1/Z, D_q of each query
  double *kw = (double *)(stats + NPAD); // [NPAD] switch values in FP64
  float *buf = (float *)(kw + NPAD);     // dO rows, then Q^T
  const int ld = kQKV * 128;
  const float inv_sqrt_d = 0.08838834764831845f;
  const int cnt = *ccount;
  // FP32: the Q rows of phase 2 are loaded during phase 1 (BF16 loads them
  // after phase 1, holding fewer registers)
  constexpr bool PREF = !BF;
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int tid = fresh_tid();
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    const int i = clist[it];
    const int n = nnei[i];
    const int base = pair_off[i];
    float4 sv[8];
    stage_rows_load<NPAD, BF>(dO, 0, 128, base, n, tid, sv);  // dO
    float gl;
    const float4 gv = gate_load(geom, base, n, tid, gl);
    const float4 av = astat[base + (tid < n ? tid : 0)];
    const int ntile = (n + 15) >> 4;
    const int kk = wave * 16 + r;
    const bool kok = kk < n;
    stage_rows_store<NPAD>(buf, tid, n, sv);
    gate_store<NPAD>(kg, kw, tid, n, gv, gl);
    if (tid < NPAD) stats[tid] = tid < n ? av : make_float4(0.f, 1.f, 0.f, 0.f);
    __syncthreads();
    float4 qpre[8];
    if constexpr (PREF) stage_t_load<NPAD, BF>(qkv, 0, ld, base, n, tid, qpre);  // Q rows of phase 2

    // ---------------- phase 1: dV, dS and the key-side sums
    floatx4 ds[NT];
    float dwk = 0.f, drkx = 0.f, drky = 0.f, drkz = 0.f;
    if (wave < ntile) {
      const float4 gk = kg[kk];
      const float wk = kok ? gk.w : 0.f;
      const double wkd = kok ? kw[kk] : 0.0;
      // lam and dA of this key against the queries of one tile (lane: key r,
      // queries 4g + v), read one query tile ahead
      const size_t col = (size_t)base * kLamLd + (kok ? kk : 0);
      const float *lc = lam + col, *dc = dA + col;
      auto lam_tile = [&](int qt, float (&lv)[4], float (&dv)[4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int qq = qt * 16 + 4 * g + v;
          const size_t off = (size_t)(qq < n ? qq : 0) * kLamLd;
          lv[v] = lc[off];
          dv[v] = dc[off];
        }
      };
      float lcur[4], lnxt[4], dcur[4], dnxt[4];
      lam_tile(0, lcur, dcur);
      floatx4 dvacc[8];
      floatx4 atp;  // BF16: A^T of the even tile of a pair
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) dvacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int qt = 0; qt < NT; ++qt) {
        ds[qt] = floatx4{0.f, 0.f, 0.f, 0.f};
        if (qt >= ntile) {
          // BF16: an unpaired last tile meets a zero partner
          if constexpr (BF)
            if (qt % 2 == 1 && qt - 1 < ntile)
              accum_rows2(buf, qt - 1, r, g, atp, floatx4{0.f, 0.f, 0.f, 0.f}, dvacc);
          continue;
        }
        if (qt + 1 < NT) lam_tile(qt + 1, lnxt, dnxt);
        floatx4 at;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int qq = qt * 16 + 4 * g + v;
          const bool ok = kok && qq < n;
          const float4 sq = stats[qq];
          const float4 gq = kg[qq];
          const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
          const float ww = gq.w * wk;
          const float lm = ok ? lcur[v] : 0.f;
          const float l = BF ? (lm + shift) * ww - shift : logit64(lm, kw[qq], wkd, shift);
          const float p = ok ? exp_hw(l - sq.x) * sq.y : 0.f;
          const float h = ww * c;
          const float dav = ok ? dcur[v] : 0.f;
          const float dH = dav * p;
          const float dL = p * (dav * h - sq.z);
          at[v] = p * h;
          ds[qt][v] = dL * ww * inv_sqrt_d;
          const float X = dL * (lm + shift) + dH * c;
          const float Y = dH * ww;
          dwk += X * gq.w;
          drkx += Y * gq.x;
          drky += Y * gq.y;
          drkz += Y * gq.z;
        }
        if constexpr (BF) {  // dV = A^T dO, tiles taken in pairs
          if (qt % 2 == 0) atp = at;
          else accum_rows2(buf, qt - 1, r, g, atp, at, dvacc);
        } else {
          accum_rows(buf, qt, r, g, at, dvacc);  // dV = A^T dO
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          lcur[v] = lnxt[v];
          dcur[v] = dnxt[v];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (kok) {
        float *dp = pt_at<BF>(dqkv, (size_t)(base + kk) * ld + 256 + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(dp, 16 * ft, dvacc[ft]);
      }
      dwk = sum_groups(dwk);
      drkx = sum_groups(drkx);
      drky = sum_groups(drky);
      drkz = sum_groups(drkz);
    }
    __syncthreads();
    if constexpr (!PREF) stage_t_load<NPAD, BF>(qkv, 0, ld, base, n, tid, qpre);
    stage_t_store<NPAD>(buf, tid, n, qpre);  // Q^T
    __syncthreads();

    // ---------------- phase 2: dK = dS^T Q
    if (wave < ntile) {
      floatx4 dkacc[8];
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) dkacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (BF) {
        // tiles in pairs; ds of tiles at or past ntile is zero
#pragma unroll
        for (int qt = 0; qt < NT; qt += 2)
          if (qt < ntile) accum_lds2<NPAD>(buf, qt, r, g, ds[qt], ds[qt + 1], dkacc);
      } else {
#pragma unroll
        for (int qt = 0; qt < NT; ++qt)
          if (qt < ntile) accum_lds<NPAD>(buf, qt, r, g, ds[qt], dkacc);
      }
      if (kok) {
        float *dp = pt_at<BF>(dqkv, (size_t)(base + kk) * ld + 128 + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(dp, 16 * ft, dkacc[ft]);
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
    __syncthreads();  // LDS is restaged for the next centre
  }
}

// ------------------------------------------------------------ fused adjoint
//
// FP32 classes of up to 96 neighbours: one workgroup per centre runs both
// halves of the adjoint.  Phase Q (wavefront = query tile) forms dA^T, the
// softmax adjoint, dS and dQ as the query-tile kernel does and leaves
// A = P H and dS of the centre in LDS ([query][key], row stride NPAD + 4),
// with the query-side sums and the key-side sums reduced over its 16
// queries; phase K (wavefront = key tile) forms dV = A^T dO and dK = dS^T Q
// from them.  Against the two-kernel form the centre's logits and gate
// records are read once, and dA and the per-pair statistics never go to
// memory.  dQ, dK and dV are accumulated in the same order as there; only
// the key-side sums are added in another order.
template <int NPAD>
constexpr int fused_ld() { return NPAD + 4; }

template <int NPAD>
size_t bwdf_lds() {
  constexpr int W = NPAD / 16;
  return sizeof(float4) * NPAD * (2 + W)  // kg, qside, key-side sums per query tile
         + sizeof(double) * NPAD          // kw
         + sizeof(float) * stage_floats<NPAD>() + sizeof(float) * 2 * NPAD * fused_ld<NPAD>();
}

// Sum of 16 per-lane values over the 16 lanes of a lane group (those that
// share lane / 16): after four halving steps lane r of the group holds the
// total of value r (30 exchanges instead of 64).  Both halves are exchanged
// and the lane keeps one sum: a select between two array elements would be
// turned into an indexed access and push the array out of registers.
__device__ __forceinline__ float reduce16_transposed(float (&v)[16], int r) {
#pragma unroll
  for (int s = 8; s >= 1; s >>= 1) {
    const bool up = (r & s) != 0;
#pragma unroll
    for (int j = 0; j < s; ++j) {
      const float lo = v[j], hi = v[j + s];
      const float lo_t = lo + __shfl_xor(lo, s);
      const float hi_t = hi + __shfl_xor(hi, s);
      v[j] = up ? hi_t : lo_t;
    }
  }
  return v[0];
}

// BF: BF16 matrix-core operands (tiles taken in pairs, every class has an
// even number) and BF16 storage of QKV, dO and dQKV, as in the two-kernel
// form; LDS and the elementwise work stay FP32.
template <int NPAD, bool BF>
__global__ __launch_bounds__(NPAD / 16 * 64, NPAD <= 64 ? 2 : 1) void k_attn_bwd_f(
    const float *__restrict__ qkv, const float *__restrict__ dO,
    const float *__restrict__ geom, const int *__restrict__ pair_off,
    const int *__restrict__ nnei, const int *__restrict__ clist, const int *__restrict__ ccount,
    int sel, float shift, const float *__restrict__ lam, const float2 *__restrict__ fstat,
    float *__restrict__ dqkv, float *__restrict__ gw, float *__restrict__ gr, int accumulate) {
  constexpr int NT = NPAD / 16;
  constexpr int LDF = fused_ld<NPAD>();
  extern __shared__ float4 smem[];
  float4 *kg = smem;                       // [NPAD] rhat, sw
  float4 *qside = kg + NPAD;               // [NPAD] query-side sums of each neighbour
  float4 *ksum = qside + NPAD;             // [NT][NPAD] key-side sums, per query tile
  double *kw = (double *)(ksum + NT * NPAD);  // [NPAD] switch values in FP64
  float *buf = (float *)(kw + NPAD);       // V rows, K^T, dO rows, Q^T in turn
  float *As = buf + stage_floats<NPAD>();  // [NPAD][LDF] A = P H
  float *Ds = As + NPAD * LDF;             // [NPAD][LDF] dS
  const int ld = kQKV * 128;
  const float inv_sqrt_d = 0.08838834764831845f;
  const int cnt = *ccount;
  // the V rows and gate records of a centre are loaded during the dK
  // product of the previous one
  float4 sv[8];
  float4 gv;
  float gl = 0.f;
  int n_nx = 0, base_nx = 0;
  if ((int)blockIdx.x < cnt) {
    const int tid = fresh_tid();
    const int i0 = clist[blockIdx.x];
    n_nx = nnei[i0];
    base_nx = pair_off[i0];
    stage_rows_load<NPAD, BF>(qkv, 256, ld, base_nx, n_nx, tid, sv);  // V
    gv = gate_load(geom, base_nx, n_nx, tid, gl);
  }
  for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int tid = fresh_tid();
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    const int n = n_nx;
    const int base = base_nx;
    const int ntile = (n + 15) >> 4;
    const int q = wave * 16 + r;
    const bool qok = q < n;
    floatx4 dov[8];
    load_rows<BF>(dO, 0, 128, base, n, q, g, dov);
    stage_rows_store<NPAD>(buf, tid, n, sv);
    gate_store<NPAD>(kg, kw, tid, n, gv, gl);
    __syncthreads();

    // ---------------- phase Q: dA^T, dS, dQ, A and dS to LDS, both sides' sums
    float4 kpre[8];  // K, read while dA^T is formed
    stage_t_load<NPAD, BF>(qkv, 128, ld, base, n, tid, kpre);
    floatx4 da[NT];
    if (wave < ntile) qk_lds<NT, BF>(buf, r, g, dov, da);  // lane: query r, keys 4g + v
    __syncthreads();
    stage_t_store<NPAD>(buf, tid, n, kpre);  // K^T
    __syncthreads();
    if (wave < ntile) {
      const int qr = qok ? q : 0;
      const float4 gq = kg[q];
      const float wq = qok ? gq.w : 0.f;
      const double wqd = qok ? kw[q] : 0.0;
      const float2 fs = fstat[base + qr];
      const float m = fs.x, invz = fs.y;
      const float *lp = lam + (size_t)(base + qr) * kLamLd + 4 * g;
      // pass 1: probabilities P (kept in registers) and logits lam (to Ds) of the
      // query's row, and D_q = sum_k P H dA (= dO . o, without o)
      float dq = 0.f;
      floatx4 pk[NT];  // P of the query's row (pass 1 -> pass 2)
      {
        floatx4 lcur = *(const floatx4 *)lp, lnxt;
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) {
          if (kt + 1 < NT) lnxt = *(const floatx4 *)(lp + 16 * (kt + 1));
          floatx4 lv;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int k = kt * 16 + 4 * g + v;
            const bool ok = qok && k < n;
            const float4 gk = kg[k];
            const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
            const float lm = ok ? lcur[v] : 0.f;
            const float l = BF ? (lm + shift) * (wq * gk.w) - shift : logit64(lm, wqd, kw[k], shift);
            const float p = ok ? exp_hw(l - m) * invz : 0.f;
            dq += p * (wq * gk.w * c) * da[kt][v];
            pk[kt][v] = p;
            lv[v] = lm;
          }
          *(floatx4 *)(Ds + q * LDF + kt * 16 + 4 * g) = lv;
          lcur = lnxt;
        }
        dq = sum_groups(dq);
      }
      floatx4 dqacc[8];
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) dqacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
      float dwq = 0.f, drqx = 0.f, drqy = 0.f, drqz = 0.f;
      floatx4 dsp;  // BF16: dS of the even tile of a pair
      // pass 2: the softmax adjoint; A = P H and dS replace P and lam
#pragma unroll
      for (int kt = 0; kt < NT; ++kt) {
        const floatx4 pv = pk[kt];
        const floatx4 lv = *(const floatx4 *)(Ds + q * LDF + kt * 16 + 4 * g);
        floatx4 ds, at;
        float ks[16];  // key-side terms: X w_q, Y rhat_q (x, y, z) for the four keys
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = kt * 16 + 4 * g + v;
          const float4 gk = kg[k];
          const float c = gq.x * gk.x + gq.y * gk.y + gq.z * gk.z;
          const float ww = wq * gk.w;
          const float lm = lv[v];
          const float p = pv[v];
          const float h = ww * c;
          const float dH = da[kt][v] * p;
          const float dL = p * (da[kt][v] * h - dq);
          ds[v] = dL * ww * inv_sqrt_d;
          at[v] = p * h;
          const float X = dL * (lm + shift) + dH * c;
          const float Y = dH * ww;
          dwq += X * gk.w;
          drqx += Y * gk.x;
          drqy += Y * gk.y;
          drqz += Y * gk.z;
          ks[v] = X * wq;
          ks[4 + v] = Y * gq.x;
          ks[8 + v] = Y * gq.y;
          ks[12 + v] = Y * gq.z;
        }
        *(floatx4 *)(As + q * LDF + kt * 16 + 4 * g) = at;
        *(floatx4 *)(Ds + q * LDF + kt * 16 + 4 * g) = ds;
        // lane r now holds the wavefront's total of term r / 4 for key
        // 4g + r % 4 of this tile
        const float kt_sum = reduce16_transposed(ks, r);
        ((float *)ksum)[(wave * NPAD + kt * 16 + 4 * g + (r & 3)) * 4 + (r >> 2)] = kt_sum;
        if constexpr (BF) {  // dQ = dS K, tiles taken in pairs
          if (kt % 2 == 0) dsp = ds;
          else accum_lds2<NPAD>(buf, kt - 1, r, g, dsp, ds, dqacc);
        } else {
          accum_lds<NPAD>(buf, kt, r, g, ds, dqacc);  // dQ = dS K
        }
      }
      dwq = sum_groups(dwq);
      drqx = sum_groups(drqx);
      drqy = sum_groups(drqy);
      drqz = sum_groups(drqz);
      if (g == 0 && qok) qside[q] = make_float4(dwq, drqx, drqy, drqz);
      if (qok) {
        float *dp = pt_at<BF>(dqkv, (size_t)(base + q) * ld + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(dp, 16 * ft, dqacc[ft]);
      }
    }
    __syncthreads();
    {
      // dO rows for phase K: each wavefront writes the rows it holds (zeros
      // past n) instead of reading them from memory a second time
      float *xr = buf + q * kLDR + 4 * g;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        *(floatx4 *)(xr + 16 * c) = qok ? dov[c] : floatx4{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();

    // ---------------- phase K: dV = A^T dO, dK = dS^T Q, key-side sums
    float4 qpre[8];  // Q, read while dV is formed
    stage_t_load<NPAD, BF>(qkv, 0, ld, base, n, tid, qpre);
    const int kk = wave * 16 + r;
    const bool kok = kk < n;
    if (wave < ntile) {
      floatx4 dvacc[8];
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) dvacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
      floatx4 atp;  // BF16: A^T of the even tile of a pair
#pragma unroll
      for (int qt = 0; qt < NT; ++qt) {
        if (qt >= ntile) {
          // BF16: an unpaired last tile meets a zero partner
          if constexpr (BF)
            if (qt % 2 == 1 && qt - 1 < ntile)
              accum_rows2(buf, qt - 1, r, g, atp, floatx4{0.f, 0.f, 0.f, 0.f}, dvacc);
          continue;
        }
        floatx4 at;  // lane: key r, queries 4g + v
#pragma unroll
        for (int v = 0; v < 4; ++v) at[v] = As[(qt * 16 + 4 * g + v) * LDF + kk];
        if constexpr (BF) {
          if (qt % 2 == 0) atp = at;
          else accum_rows2(buf, qt - 1, r, g, atp, at, dvacc);
        } else {
          accum_rows(buf, qt, r, g, at, dvacc);
        }
      }
      if (kok) {
        float *dp = pt_at<BF>(dqkv, (size_t)(base + kk) * ld + 256 + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(dp, 16 * ft, dvacc[ft]);
      }
    }
    __syncthreads();
    stage_t_store<NPAD>(buf, tid, n, qpre);  // Q^T
    __syncthreads();
    {
      const int itn = it + (int)gridDim.x;
      if (itn < cnt) {
        const int inx = clist[itn];
        n_nx = nnei[inx];
        base_nx = pair_off[inx];
        stage_rows_load<NPAD, BF>(qkv, 256, ld, base_nx, n_nx, tid, sv);  // next V
        gv = gate_load(geom, base_nx, n_nx, tid, gl);
      }
    }
    if (wave < ntile) {
      floatx4 dkacc[8];
#pragma unroll
      for (int ft = 0; ft < 8; ++ft) dkacc[ft] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (BF) {
        // tiles in pairs; dS of query tiles at or past ntile (not written for
        // this centre) is zero
#pragma unroll
        for (int qt = 0; qt < NT; qt += 2) {
          if (qt >= ntile) continue;
          floatx4 d0, d1;
          const bool ok1 = qt + 1 < ntile;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            d0[v] = Ds[(qt * 16 + 4 * g + v) * LDF + kk];
            const float x1 = Ds[((qt + 1) * 16 + 4 * g + v) * LDF + kk];
            d1[v] = ok1 ? x1 : 0.f;
          }
          accum_lds2<NPAD>(buf, qt, r, g, d0, d1, dkacc);
        }
      } else {
#pragma unroll
        for (int qt = 0; qt < NT; ++qt) {
          if (qt >= ntile) continue;
          floatx4 dsv;
#pragma unroll
          for (int v = 0; v < 4; ++v) dsv[v] = Ds[(qt * 16 + 4 * g + v) * LDF + kk];
          accum_lds<NPAD>(buf, qt, r, g, dsv, dkacc);
        }
      }
      if (kok) {
        float *dp = pt_at<BF>(dqkv, (size_t)(base + kk) * ld + 128 + 4 * g);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) stp4<BF>(dp, 16 * ft, dkacc[ft]);
        if (g == 0) {
          float4 t = qside[kk];
          for (int w = 0; w < ntile; ++w) {
            const float4 kv = ksum[w * NPAD + kk];
            t.x += kv.x;
            t.y += kv.y;
            t.z += kv.z;
            t.w += kv.w;
          }
          const size_t p = (size_t)(base + kk);
          if (accumulate) {
            gw[p] += t.x;
            gr[4 * p + 0] += t.y;
            gr[4 * p + 1] += t.z;
            gr[4 * p + 2] += t.w;
          } else {
            gw[p] = t.x;
            gr[4 * p + 0] = t.y;
            gr[4 * p + 1] = t.z;
            gr[4 * p + 2] = t.w;
            gr[4 * p + 3] = 0.f;
          }
        }
      }
    }
    __syncthreads();  // LDS is restaged for the next centre
  }
}

// Class lists: centre i with n = nnei[i] > 0 belongs to class (n - 1) / 32
// (counted in ccount[4 + class]) and is listed in the smallest class of the
// active set (bit c of `active`) that holds n neighbours; the host keeps the
// top class active, so every centre is listed.  A class that is not active
// is not launched: the host deactivates classes that were empty in an
// earlier step, and a centre that falls into one after all is computed by
// the next larger active class (more padding, the same result: the host
// keeps the largest class of the fused FP32 adjoint active, so the fallback
// never changes the kind of adjoint).  Positions
// are taken with one atomic per wavefront and class, so the order inside a
// list varies from run to run; every centre is computed on its own, so
// results do not depend on it.
__global__ void k_attn_classes(const int *__restrict__ nnei, int nloc, int active,
                               int *__restrict__ ccount, int *__restrict__ clist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int n = i < nloc ? nnei[i] : 0;
  const int nat = n > 0 ? (n - 1) >> 5 : -1;
  int cls = nat;
  if (cls >= 0)
    while (cls < 3 && !((active >> cls) & 1)) ++cls;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const unsigned long long bn = __ballot(nat == c);
    if (bn != 0ull && lane == __ffsll((long long)bn) - 1) atomicAdd(&ccount[4 + c], __popcll(bn));
    const unsigned long long b = __ballot(cls == c);
    if (b == 0ull) continue;
    const int leader = __ffsll((long long)b) - 1;
    int pos0 = 0;
    if (lane == leader) pos0 = atomicAdd(&ccount[c], __popcll(b));
    pos0 = __shfl(pos0, leader);
    if (cls == c) clist[(size_t)c * nloc + pos0 + __popcll(b & ((1ull << lane) - 1ull))] = i;
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
// KF features per lane (16 lanes x KF >= ldg); LN_MODE as ln_mode below, fixed
// at compile time so that operands a mode does not use are never loaded.
template <int KF, int LN_MODE>
__global__ __launch_bounds__(256) void k_desc_bwd(
    const float *__restrict__ geom, const float *__restrict__ G, int ldg,
    const float *__restrict__ T, const float *__restrict__ dD, int ldd,
    const int *__restrict__ pair_off, const int *__restrict__ nnei, int sel, int M, int axis,
    const float *__restrict__ gamma, const float *__restrict__ xhat,
    const float *__restrict__ rstd, const float *__restrict__ temb, float *__restrict__ dG,
    float *__restrict__ dnext, float *__restrict__ dRt) {
  constexpr int ln_mode = LN_MODE;
  __shared__ float Ts[4][128];
  __shared__ float dTs[4][128];
  __shared__ float part[16][16][4];
  __shared__ float gam[128];  // gamma of the layer norm (ln_mode 0), zeros past M
  const int i = blockIdx.x;
  const int n = nnei[i];
  const int base = pair_off[i];
  const int tid = threadIdx.x;
  if (tid < 128) {
    for (int c = 0; c < 4; ++c) Ts[c][tid] = tid < M ? T[(size_t)i * 4 * M + c * M + tid] : 0.f;
    gam[tid] = (ln_mode == 0 && tid < M) ? gamma[tid] : 0.f;
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
  // Every global load of a pair is issued before any of its values is used
  // and is unconditional: feature indices are clamped to the row (columns
  // past M hold zeros).
  for (int j = grp; j < n; j += 16) {
    const size_t p = (size_t)(base + j);
    const float4 gq = *(const float4 *)(geom + p * kGeom);  // s, rx, ry, rz
    float gm[KF], xv[KF], tv[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int m = li + 16 * k;
      const int mc = m < ldg ? m : 0;
      gm[k] = G[p * ldg + mc];
      xv[k] = ln_mode == 0 ? xhat[p * ldg + mc] : 0.f;
      tv[k] = ln_mode == 1 ? temb[p * ldg + mc] : 0.f;
    }
    const float rs = ln_mode == 0 ? rstd[p] : 0.f;
    const float R0 = gq.x, R1 = gq.x * gq.y, R2 = gq.x * gq.z, R3 = gq.x * gq.w;
    float dg[KF];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int m = li + 16 * k;
      const int mc = m < 128 ? m : 0;
      const bool in = m < M;
      const float v = R0 * dTs[0][mc] + R1 * dTs[1][mc] + R2 * dTs[2][mc] + R3 * dTs[3][mc];
      const float gmv = in ? gm[k] : 0.f;
      dg[k] = in ? v : 0.f;
      a0 += gmv * dTs[0][mc];
      a1 += gmv * dTs[1][mc];
      a2 += gmv * dTs[2][mc];
      a3 += gmv * dTs[3][mc];
      const float dx = gam[mc] * dg[k];
      s1 += dx;
      s2 += in ? dx * xv[k] : 0.f;
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
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int m = li + 16 * k;
      if (m < ldg) {
        const int mc = m < 128 ? m : 0;
        const float ln = rs * (gam[mc] * dg[k] - s1 * invm - xv[k] * s2 * invm);
        const float th = dg[k] * (1.0f - tv[k] * tv[k]);
        const float nx = m < M ? (ln_mode == 0 ? ln : th) : 0.f;
        dG[p * ldg + m] = dg[k];
        if (ln_mode != 2) dnext[p * ldg + m] = nx;
      }
    }
    if (li == 0) *(float4 *)(dRt + 4 * p) = make_float4(a0, a1, a2, a3);
  }
}

// The descriptor adjoint fused with the adjoint of the last attention
// layer's output projection (Sec. II-B, DPA-1).  Per centre dT is formed as
// in k_desc_bwd; then each wavefront takes 16-neighbour tiles and forms, per
// pair, the residual-path gradient dG = R~ dT / sel, dR~ = dT G / sel, the
// layer-norm adjoint d(acc) of the pre-norm projection output, and finally
// dO = d(acc) W_O^T on the matrix cores with W_O^T resident in LDS.  d(acc)
// is produced in registers already in the operand layout of that product
// (lane l: pair l % 16, features 16 c + 4 (l / 16) + {0..3}), so it never
// reaches memory.  Blocks walk over centres (persistent grid), so W_O^T is
// staged once per workgroup.
//
// Shape: ldg = 112 (seven 16-feature chunks) and 96 < M <= 100, so the last
// chunk holds M - 96 real features: lane group g carries feature 96 + g of
// it, in one matrix-core step of depth four (FP32) or in the first operand
// slot of the last chunk pair (BF16).
constexpr int kDoN = 128;            // attention width: rows of W_O^T, columns of dO
constexpr int kDoK = 112;            // padded feature width of G
constexpr int kDoLdw = kDoK + 4;     // LDS row stride of W_O^T
constexpr int kDoDs = 17;            // LDS row stride of a centre's dD (axis <= 16)
constexpr int kDoLds = kDoN * kDoLdw + 4 * 128 * 2 + 16 * 16 * 4 + 128 + 1712;  // floats

struct DescOprojArgs {
  const float *geom, *G, *T, *dD;
  const int *pair_off, *nnei;
  int nloc, sel, M, axis, ldd;
  const float *gamma, *xhat, *rstd;
  const float *Wt;  // [kDoN][kDoK]: W_O^T of the last attention layer
  float *dG, *dRt;
  float *dO;        // [pairs][kDoN]: FP32, or BF16 (rounded to nearest even) when BF
};

template <bool BF>
__global__ __launch_bounds__(256, 2) void k_desc_oproj_bwd(DescOprojArgs a) {
  extern __shared__ float sm[];
  float *wsm = sm;                        // [kDoN][kDoLdw]
  float *Ts = wsm + kDoN * kDoLdw;        // [4][128]
  float *dTs = Ts + 4 * 128;              // [4][128]
  float *part = dTs + 4 * 128;            // [16][16][4]
  float *gam = part + 16 * 16 * 4;        // [128], zeros past M
  float *dDs = gam + 128;                 // [M][kDoDs]: the centre's dD
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int M = a.M, axis = a.axis;
  for (int idx = tid; idx < kDoN * (kDoK / 4); idx += 256) {
    const int n = idx / (kDoK / 4), c4 = idx % (kDoK / 4);
    *(float4 *)(wsm + n * kDoLdw + 4 * c4) = *(const float4 *)(a.Wt + (size_t)n * kDoK + 4 * c4);
  }
  if (tid < 128) gam[tid] = tid < M ? a.gamma[tid] : 0.f;
  const float inv = 1.0f / (float)a.sel;
  const float invm = 1.0f / (float)M;
  const int f6 = 96 + g;                  // this lane's feature of the last chunk
  const bool in6 = f6 < M;
  // A centre's dD row (ldd <= 512 float4) and T column tid arrive in
  // registers one centre ahead (issued while the current centre's tiles run)
  // and are then staged in LDS.
  const int nq = a.ldd >> 2;
  float4 dq[2];
  float tq[4];
  auto fetch = [&](int i) {
    const float4 *src = (const float4 *)(a.dD + (size_t)i * a.ldd);
    dq[0] = src[tid < nq ? tid : 0];
    dq[1] = src[tid + 256 < nq ? tid + 256 : 0];
    const float *tp = a.T + (size_t)i * 4 * M + (tid < M ? tid : 0);
#pragma unroll
    for (int c = 0; c < 4; ++c) tq[c] = tp[c * M];
  };
  // One tile's pair rows (rows past n read the centre's first pair).  A
  // wavefront issues its first tile of a centre before the centre's dT is
  // formed and each next tile while the current one is on the matrix cores.
  floatx4 gv[6], xv[6];
  float g6, x6, rs;
  float4 gq;
  auto load_tile = [&](int t, int base, int n) {
    const int j = 16 * t + r;
    const size_t p = (size_t)base + (j < n ? j : 0);
    gq = *(const float4 *)(a.geom + p * kGeom);  // s, rx, ry, rz
    rs = a.rstd[p];
    const float *gp = a.G + p * kDoK + 4 * g;
    const float *xp = a.xhat + p * kDoK + 4 * g;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      gv[c] = *(const floatx4 *)(gp + 16 * c);
      xv[c] = *(const floatx4 *)(xp + 16 * c);
    }
    g6 = a.G[p * kDoK + f6];
    x6 = a.xhat[p * kDoK + f6];
  };
  if (blockIdx.x < a.nloc) fetch(blockIdx.x);
  for (int i = blockIdx.x; i < a.nloc; i += gridDim.x) {
    const int n = a.nnei[i];
    const int base = a.pair_off[i];
    const int ntile = (n + 15) >> 4;
    if (wave < ntile) load_tile(wave, base, n);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int q = tid + 256 * k;
      if (q < nq) {
        const float v4[4] = {dq[k].x, dq[k].y, dq[k].z, dq[k].w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = 4 * q + v, m = e / axis;
          if (m < M) dDs[m * kDoDs + (e - m * axis)] = v4[v];
        }
      }
    }
    if (tid < 128)
#pragma unroll
      for (int c = 0; c < 4; ++c) Ts[c * 128 + tid] = tid < M ? tq[c] : 0.f;
    __syncthreads();  // also: every wavefront is done with the previous centre's dTs
    if (i + (int)gridDim.x < a.nloc) fetch(i + gridDim.x);
    {
      const int aa = tid & 15, pp = tid >> 4;
      float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
      if (aa < axis) {
        for (int mm = pp; mm < M; mm += 16) {
          const float x = dDs[mm * kDoDs + aa];
          q0 += x * Ts[0 * 128 + mm];
          q1 += x * Ts[1 * 128 + mm];
          q2 += x * Ts[2 * 128 + mm];
          q3 += x * Ts[3 * 128 + mm];
        }
      }
      *(float4 *)(part + (pp * 16 + aa) * 4) = make_float4(q0, q1, q2, q3);
    }
    __syncthreads();
    if (tid < 128) {
      float d0 = 0.f, d1 = 0.f, d2 = 0.f, d3 = 0.f;
      if (tid < M) {
        for (int c = 0; c < axis; ++c) {
          const float x = dDs[tid * kDoDs + c];
          d0 += x * Ts[0 * 128 + c];
          d1 += x * Ts[1 * 128 + c];
          d2 += x * Ts[2 * 128 + c];
          d3 += x * Ts[3 * 128 + c];
        }
        if (tid < axis && tid < 16) {
          for (int pp = 0; pp < 16; ++pp) {
            const float4 q = *(const float4 *)(part + (pp * 16 + tid) * 4);
            d0 += q.x;
            d1 += q.y;
            d2 += q.z;
            d3 += q.w;
          }
        }
      }
      dTs[0 * 128 + tid] = d0 * inv;
      dTs[1 * 128 + tid] = d1 * inv;
      dTs[2 * 128 + tid] = d2 * inv;
      dTs[3 * 128 + tid] = d3 * inv;
    }
    __syncthreads();
    for (int t = wave; t < ntile; t += 4) {
      const int j = 16 * t + r;
      const bool ok = j < n;
      const size_t p = (size_t)base + (ok ? j : 0);
      const float R0 = gq.x, R1 = gq.x * gq.y, R2 = gq.x * gq.z, R3 = gq.x * gq.w;
      floatx4 dy[6];
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int f = 16 * c + 4 * g;
        const floatx4 t0 = *(const floatx4 *)(dTs + 0 * 128 + f);
        const floatx4 t1 = *(const floatx4 *)(dTs + 1 * 128 + f);
        const floatx4 t2 = *(const floatx4 *)(dTs + 2 * 128 + f);
        const floatx4 t3 = *(const floatx4 *)(dTs + 3 * 128 + f);
        const floatx4 gm = *(const floatx4 *)(gam + f);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          dy[c][v] = R0 * t0[v] + R1 * t1[v] + R2 * t2[v] + R3 * t3[v];
          a0 += gv[c][v] * t0[v];
          a1 += gv[c][v] * t1[v];
          a2 += gv[c][v] * t2[v];
          a3 += gv[c][v] * t3[v];
          const float dx = gm[v] * dy[c][v];
          s1 += dx;
          s2 += dx * xv[c][v];
        }
      }
      float dy6;
      {
        const float t0 = dTs[0 * 128 + f6], t1 = dTs[1 * 128 + f6];
        const float t2 = dTs[2 * 128 + f6], t3 = dTs[3 * 128 + f6];
        const float gmv = in6 ? g6 : 0.f;
        dy6 = in6 ? R0 * t0 + R1 * t1 + R2 * t2 + R3 * t3 : 0.f;
        a0 += gmv * t0;
        a1 += gmv * t1;
        a2 += gmv * t2;
        a3 += gmv * t3;
        const float dx = gam[f6] * dy6;
        s1 += dx;
        s2 += in6 ? dx * x6 : 0.f;
      }
      a0 = sum_groups(a0);
      a1 = sum_groups(a1);
      a2 = sum_groups(a2);
      a3 = sum_groups(a3);
      s1 = sum_groups(s1);
      s2 = sum_groups(s2);
      if (ok) {
        float *dgp = a.dG + p * kDoK;
#pragma unroll
        for (int c = 0; c < 6; ++c) *(floatx4 *)(dgp + 16 * c + 4 * g) = dy[c];
        dgp[f6] = dy6;
        if (g > 0) *(floatx4 *)(dgp + 96 + 4 * g) = floatx4{0.f, 0.f, 0.f, 0.f};  // 100..111
        if (g == 0) *(float4 *)(a.dRt + 4 * p) = make_float4(a0, a1, a2, a3);
      }
      // layer-norm adjoint, in place of dy
      const float m1 = s1 * invm, m2 = s2 * invm;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const floatx4 gm = *(const floatx4 *)(gam + 16 * c + 4 * g);
#pragma unroll
        for (int v = 0; v < 4; ++v) dy[c][v] = rs * (gm[v] * dy[c][v] - m1 - xv[c][v] * m2);
      }
      const float x6a = in6 ? rs * (gam[f6] * dy6 - m1 - x6 * m2) : 0.f;
      if (t + 4 < ntile) load_tile(t + 4, base, n);
      floatx4 acc[8];
#pragma unroll
      for (int nt = 0; nt < 8; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
      // the weight offsets are laundered per tile so that the compiler does
      // not hoist all of W_O^T into registers across tiles
      int woff = r * kDoLdw + 4 * g, w6off = r * kDoLdw + f6;
      asm volatile("" : "+v"(woff), "+v"(w6off));
      const float *wl = wsm + woff;
      if constexpr (BF) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const bf16x8 xb = to_bf16x8(dy[2 * q], dy[2 * q + 1]);
#pragma unroll
          for (int nt = 0; nt < 8; ++nt) {
            const floatx4 w0 = *(const floatx4 *)(wl + nt * 16 * kDoLdw + 32 * q);
            const floatx4 w1 = *(const floatx4 *)(wl + nt * 16 * kDoLdw + 32 * q + 16);
            acc[nt] = mfma_bf16x2(to_bf16x8(w0, w1), xb, acc[nt]);
          }
        }
        const floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
        const bf16x8 xb = to_bf16x8(floatx4{x6a, 0.f, 0.f, 0.f}, z);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
          const float w6 = wsm[w6off + nt * 16 * kDoLdw];
          acc[nt] = mfma_bf16x2(to_bf16x8(floatx4{w6, 0.f, 0.f, 0.f}, z), xb, acc[nt]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          floatx4 w[8];
#pragma unroll
          for (int nt = 0; nt < 8; ++nt) w[nt] = *(const floatx4 *)(wl + nt * 16 * kDoLdw + 16 * c);
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) acc[nt] = mfma4(w[nt][v], dy[c][v], acc[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
          acc[nt] = mfma4(wsm[w6off + nt * 16 * kDoLdw], x6a, acc[nt]);
      }
      if (ok) {
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
          const size_t o = p * kDoN + nt * 16 + 4 * g;
          if constexpr (BF)
            *(bf16x4 *)((__bf16 *)a.dO + o) = to_bf16(acc[nt]);
          else
            *(floatx4 *)(a.dO + o) = acc[nt];
        }
      }
    }
  }
}

// Centres are grouped by neighbour count into classes of 32, 64, 96 and 128
// slots; each class runs a kernel sized for it, over its own centre list, so
// the common case does not pay for the largest LDS size and an empty class
// costs one wave of exiting blocks.
template <int NPAD, bool OP = false>
size_t fwd_lds() {
  return (sizeof(float4) + sizeof(double)) * NPAD + sizeof(float) * stage_floats<NPAD>() +
         (OP ? sizeof(float) * (kOpCols * kLDR + 3 * kOpCols) : 0);
}
template <int NPAD>
size_t bwdq_lds() {
  return (sizeof(float4) + sizeof(double)) * NPAD + sizeof(float) * stage_floats<NPAD>();
}
template <int NPAD>
size_t bwdk_lds() {
  return (sizeof(float4) * 2 + sizeof(double)) * NPAD + sizeof(float) * stage_floats<NPAD>();
}

// Persistent grid sizes: resident blocks per CU times CUs, per device.
constexpr int kMaxDevices = 64;
int g_grid[kMaxDevices][10][4];  // fwd, bwd_q, bwd_k in FP32, then in BF16; fused FP32
                                 // adjoint; FP32 forward with the output projection; fused
                                 // BF16 adjoint; BF16 forward with the output projection

int g_desc_grid[kMaxDevices][2];  // fused descriptor / projection adjoint: FP32, BF16

// Blocks of the grid of a class that held no centres in a recent step: an
// empty launch of the full persistent grid costs ~20 us.
constexpr int kSmallGrid = 32;

int grid_for(int kind, int cls, int small = 0) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  const int gsz = g_grid[dev][kind][cls] > 0 ? g_grid[dev][kind][cls] : 1024;
  return ((small >> cls) & 1) && gsz > kSmallGrid ? kSmallGrid : gsz;
}

template <class K>
hipError_t occupancy_grid(K kernel, int threads, size_t lds, int cus, int *out) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds);
  if (e != hipSuccess) return e;
  *out = (nb > 0 ? nb : 1) * cus;
  return hipSuccess;
}

template <int NPAD, bool BF>
hipError_t prepare_class(int dev, int cus, int cls) {
  const int th = NPAD / 16 * 64;
  const int k0 = BF ? 3 : 0;  // grid table rows: fp32 fwd, bwd_q, bwd_k, then bf16
  hipError_t e = hipSuccess;
  if (NPAD > 64) {
    e = hipFuncSetAttribute((const void *)k_attn_fwd<NPAD, BF, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_lds<NPAD>());
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_attn_bwd_q<NPAD, BF>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwdq_lds<NPAD>());
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_attn_bwd_k<NPAD, BF>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwdk_lds<NPAD>());
  }
  if (e == hipSuccess)
    e = occupancy_grid(k_attn_fwd<NPAD, BF, false>, th, fwd_lds<NPAD>(), cus,
                       &g_grid[dev][k0][cls]);
  if (e == hipSuccess)
    e = occupancy_grid(k_attn_bwd_q<NPAD, BF>, th, bwdq_lds<NPAD>(), cus,
                       &g_grid[dev][k0 + 1][cls]);
  if (e == hipSuccess)
    e = occupancy_grid(k_attn_bwd_k<NPAD, BF>, th, bwdk_lds<NPAD>(), cus,
                       &g_grid[dev][k0 + 2][cls]);
  if (e == hipSuccess && fwd_lds<NPAD, true>() > 65536)
    e = hipFuncSetAttribute((const void *)k_attn_fwd<NPAD, BF, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_lds<NPAD, true>());
  if (e == hipSuccess)
    e = occupancy_grid(k_attn_fwd<NPAD, BF, true>, th, fwd_lds<NPAD, true>(), cus,
                       &g_grid[dev][BF ? 9 : 7][cls]);
  if constexpr (NPAD <= 96) {
    if (e == hipSuccess && bwdf_lds<NPAD>() > 65536)
      e = hipFuncSetAttribute((const void *)k_attn_bwd_f<NPAD, BF>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwdf_lds<NPAD>());
    if (e == hipSuccess)
      e = occupancy_grid(k_attn_bwd_f<NPAD, BF>, th, bwdf_lds<NPAD>(), cus,
                         &g_grid[dev][BF ? 8 : 6][cls]);
  }
  return e;
}

}  // namespace

int attn_class_count(int sel) { return sel <= 32 ? 1 : sel <= 64 ? 2 : sel <= 96 ? 3 : 4; }
int attn_class_npad(int cls) { return 32 * (cls + 1); }

hipError_t attn_prepare() {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (e == hipSuccess) e = prepare_class<32, false>(dev, cus, 0);
  if (e == hipSuccess) e = prepare_class<64, false>(dev, cus, 1);
  if (e == hipSuccess) e = prepare_class<96, false>(dev, cus, 2);
  if (e == hipSuccess) e = prepare_class<128, false>(dev, cus, 3);
  if (e == hipSuccess) e = prepare_class<32, true>(dev, cus, 0);
  if (e == hipSuccess) e = prepare_class<64, true>(dev, cus, 1);
  if (e == hipSuccess) e = prepare_class<96, true>(dev, cus, 2);
  if (e == hipSuccess) e = prepare_class<128, true>(dev, cus, 3);
  const int lds = (int)(sizeof(float) * kDoLds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_desc_oproj_bwd<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_desc_oproj_bwd<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = occupancy_grid(k_desc_oproj_bwd<false>, 256, lds, cus, &g_desc_grid[dev][0]);
  if (e == hipSuccess)
    e = occupancy_grid(k_desc_oproj_bwd<true>, 256, lds, cus, &g_desc_grid[dev][1]);
  return e;
}

void launch_attn_classes(const int *nnei, int nloc, int active, int *ccount, int *clist,
                         hipStream_t s) {
  if (nloc <= 0) return;
  hipLaunchKernelGGL(k_attn_classes, dim3((nloc + 255) / 256), dim3(256), 0, s, nnei, nloc,
                     active, ccount, clist);
}

// class (compile-time NP) and precision (compile-time BFV) dispatch
#define ATTN_CLASS_SWITCH1(cls, ...)                           \
  switch (cls) {                                               \
    case 0: { constexpr int NP = 32; __VA_ARGS__; } break;     \
    case 1: { constexpr int NP = 64; __VA_ARGS__; } break;     \
    case 2: { constexpr int NP = 96; __VA_ARGS__; } break;     \
    default: { constexpr int NP = 128; __VA_ARGS__; } break;   \
  }
#define ATTN_CLASS_SWITCH(cls, ...)                            \
  if (a.bf16) {                                                \
    constexpr bool BFV = true;                                 \
    ATTN_CLASS_SWITCH1(cls, __VA_ARGS__)                       \
  } else {                                                     \
    constexpr bool BFV = false;                                \
    ATTN_CLASS_SWITCH1(cls, __VA_ARGS__)                       \
  }

void launch_attn_fwd_class(int cls, const AttnArgs &a, const float *qkv, float *out, float *lam,
                           float *fstat, const AttnOut *op, hipStream_t s) {
  if (a.nloc <= 0) return;
  const int *cl = a.clist + (size_t)cls * a.nloc, *cc = a.ccount + cls;
  if (op) {
    const dim3 grid(grid_for(a.bf16 ? 9 : 7, cls, a.small));
    ATTN_CLASS_SWITCH(cls, hipLaunchKernelGGL((k_attn_fwd<NP, BFV, true>), grid,
                                              dim3(NP / 16 * 64), (fwd_lds<NP, true>()), s, qkv,
                                              a.geom, a.pair_off, a.nnei, cl, cc, a.sel, a.shift,
                                              out, lam, (float2 *)fstat, *op));
    return;
  }
  const dim3 grid(grid_for(a.bf16 ? 3 : 0, cls, a.small));
  ATTN_CLASS_SWITCH(cls, hipLaunchKernelGGL((k_attn_fwd<NP, BFV, false>), grid, dim3(NP / 16 * 64),
                                            fwd_lds<NP>(), s, qkv, a.geom, a.pair_off, a.nnei,
                                            cl, cc, a.sel, a.shift, out, lam, (float2 *)fstat,
                                            AttnOut{}));
}

void launch_attn_bwd_q_class(int cls, const AttnArgs &a, const float *qkv, const float *o,
                             const float *dO, const float *lam, const float *fstat, float *dqkv,
                             float *astat, float *qside, float *dA, hipStream_t s) {
  if (a.nloc <= 0) return;
  const int *cl = a.clist + (size_t)cls * a.nloc, *cc = a.ccount + cls;
  const dim3 grid(grid_for(a.bf16 ? 4 : 1, cls, a.small));
  ATTN_CLASS_SWITCH(cls, hipLaunchKernelGGL((k_attn_bwd_q<NP, BFV>), grid, dim3(NP / 16 * 64),
                                            bwdq_lds<NP>(), s, qkv, o, dO, a.geom, a.pair_off,
                                            a.nnei, cl, cc, a.sel, a.shift, lam,
                                            (const float2 *)fstat, dqkv, (float4 *)astat,
                                            (float4 *)qside, dA));
}

bool attn_bwd_fused(const AttnArgs &, int cls) { return cls <= 2; }

void launch_attn_bwd_fused_class(int cls, const AttnArgs &a, const float *qkv, const float *dO,
                                 const float *lam, const float *fstat, float *dqkv, float *gw,
                                 float *gr, int accumulate, hipStream_t s) {
  if (a.nloc <= 0 || !attn_bwd_fused(a, cls)) return;
  const int *cl = a.clist + (size_t)cls * a.nloc, *cc = a.ccount + cls;
  const dim3 grid(grid_for(a.bf16 ? 8 : 6, cls, a.small));
#define ATTN_BWD_F(NP, BFV)                                                                    \
  hipLaunchKernelGGL((k_attn_bwd_f<NP, BFV>), grid, dim3(NP / 16 * 64), bwdf_lds<NP>(), s, qkv, \
                     dO, a.geom, a.pair_off, a.nnei, cl, cc, a.sel, a.shift, lam,              \
                     (const float2 *)fstat, dqkv, gw, gr, accumulate)
  if (a.bf16) {
    if (cls == 0) ATTN_BWD_F(32, true);
    else if (cls == 1) ATTN_BWD_F(64, true);
    else ATTN_BWD_F(96, true);
  } else {
    if (cls == 0) ATTN_BWD_F(32, false);
    else if (cls == 1) ATTN_BWD_F(64, false);
    else ATTN_BWD_F(96, false);
  }
#undef ATTN_BWD_F
}

void launch_attn_bwd_k_class(int cls, const AttnArgs &a, const float *qkv, const float *dO,
                             const float *lam, const float *dA, float *dqkv, const float *astat,
                             const float *qside, float *gw, float *gr, int accumulate,
                             hipStream_t s) {
  if (a.nloc <= 0) return;
  const int *cl = a.clist + (size_t)cls * a.nloc, *cc = a.ccount + cls;
  const dim3 grid(grid_for(a.bf16 ? 5 : 2, cls, a.small));
  ATTN_CLASS_SWITCH(cls, hipLaunchKernelGGL((k_attn_bwd_k<NP, BFV>), grid, dim3(NP / 16 * 64),
                                            bwdk_lds<NP>(), s, qkv, dO, a.geom, a.pair_off,
                                            a.nnei, cl, cc, a.shift, lam, dA, dqkv,
                                            (const float4 *)astat, (const float4 *)qside, gw, gr,
                                            accumulate));
}

void launch_desc_fwd(const float *geom, const float *G, int ldg, const int *pair_off,
                     const int *nnei, int nloc, int sel, int M, int axis, float *T, float *dmat,
                     hipStream_t s) {
  if (nloc <= 0) return;
  const int ldd = pad16(M * axis);
  // one lane per feature: a single wavefront when M <= 64
  const int threads = M <= 64 ? 64 : 128;
  hipLaunchKernelGGL(k_desc_fwd, dim3(nloc), dim3(threads), 0, s, geom, G, ldg, pair_off, nnei,
                     sel, M, axis, T, dmat, ldd);
}

void launch_desc_bwd(const float *geom, const float *G, int ldg, const float *T,
                     const float *dD, const int *pair_off, const int *nnei, int nloc, int sel,
                     int M, int axis, int ln_mode, const float *gamma, const float *xhat,
                     const float *rstd, const float *t_emb, float *dG, float *dnext,
                     float *dRt, hipStream_t s) {
  if (nloc <= 0) return;
  const int ldd = pad16(M * axis);
#define DESC_BWD(KF, MODE)                                                                  \
  hipLaunchKernelGGL((k_desc_bwd<KF, MODE>), dim3(nloc), dim3(256), 0, s, geom, G, ldg, T, dD, \
                     ldd, pair_off, nnei, sel, M, axis, gamma, xhat, rstd, t_emb, dG, dnext,   \
                     dRt)
  if (ldg <= 64) {
    if (ln_mode == 0)
      DESC_BWD(4, 0);
    else if (ln_mode == 1)
      DESC_BWD(4, 1);
    else
      DESC_BWD(4, 2);
  } else {
    if (ln_mode == 0)
      DESC_BWD(8, 0);
    else if (ln_mode == 1)
      DESC_BWD(8, 1);
    else
      DESC_BWD(8, 2);
  }
#undef DESC_BWD
}

bool desc_oproj_fusable(int ldg, int M, int axis, int D) {
  return ldg == kDoK && M > 96 && M <= 100 && axis >= 1 && axis <= 16 && D == kDoN;
}

void launch_desc_oproj_bwd(const float *geom, const float *G, const float *T, const float *dD,
                           const int *pair_off, const int *nnei, int nloc, int sel, int M,
                           int axis, const float *gamma, const float *xhat, const float *rstd,
                           const float *Wt, float *dG, float *dRt, float *dO, int bf16,
                           hipStream_t s) {
  if (nloc <= 0) return;
  const DescOprojArgs a{geom, G,     T,         dD,   pair_off, nnei, nloc, sel,
                        M,    axis,  pad16(M * axis), gamma, xhat, rstd, Wt,  dG,
                        dRt,  dO};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  int grid = g_desc_grid[dev][bf16 ? 1 : 0];
  if (grid <= 0) grid = 512;
  if (grid > nloc) grid = nloc;
  const size_t lds = sizeof(float) * kDoLds;
  if (bf16)
    hipLaunchKernelGGL(k_desc_oproj_bwd<true>, dim3(grid), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL(k_desc_oproj_bwd<false>, dim3(grid), dim3(256), lds, s, a);
}

}  // namespace dpa1
