// Fused embedding net (layers 2 and 3) forward, and its input-gradient
// adjoint with recomputation, for the three-layer type-embedded embedding net
// of DPA-1 (Sec. II-B: the embedding matrix G carries the type embedding).
//
// The first layer h1 = tanh(table[t_j][t_i] + ws * s) is produced per pair by
// the geometry kernel.  Here one wavefront takes 32 pairs through
//   h2 = tanh(h1 W2 + b2) + res(h1),   G0 = tanh(h2 W3 + b3) + res(h2)
// on v_mfma_f32_16x16x4_f32 with the transposed-product layout (each lane
// holds four consecutive columns of one row), in which the output of one
// layer is already the B operand of the next, so nothing but the residual
// lookups leaves the registers.  The adjoint recomputes h2 and the tanh
// outputs from h1 instead of storing them, and ends with the scalar
// dE/ds = sum_o dE/du1[o] * ws[o] per pair.
#include <type_traits>

#include "dpa1_internal.h"

namespace dpa1 {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 precision mode: one gfx950 v_mfma_f32_16x16x32_bf16 per pair of
// 16-wide k chunks, each lane's eight operand slots holding its four
// consecutive k of the first chunk and then of the second (on both operands
// alike: the sum of two 16x16x16 steps); a lone last chunk is paired with
// zeros.  FP32 accumulation.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x4 to_bf16(const floatx4 &v) {
  return __builtin_convertvector(v, bf16x4);
}
__device__ __forceinline__ bf16x8 to_bf16x8(const floatx4 &lo, const floatx4 &hi) {
  return __builtin_shufflevector(to_bf16(lo), to_bf16(hi), 0, 1, 2, 3, 4, 5, 6, 7);
}

// acc[mt][nt] = sum_k W[nt*16 + r][k] x[mt][k] over the wavefront's MT 16-row
// tiles (W row-major [NTILE*16][LDW], in global memory or in LDS).
// KT < 4 (FP32 only): x and W hold data only in the first 4 KT columns of the
// last 16-wide chunk (zeros past them), which then takes KT MFMA steps
// instead of four: in step s lane group g carries depth 16 (KCH - 1) + 4 s + g
// on both operands (W loaded at that depth, x taken from the lane that holds
// it: lane r + 16 s, element g).
template <int KCH, int NTILE, bool BF, int KT, int LDW = KCH * 16, int MT, typename WT>
__device__ __forceinline__ void layer(const WT *__restrict__ W, int r, int g,
                                      const floatx4 (&x)[MT][KCH], floatx4 (&acc)[MT][NTILE]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < KCH; ++c) {
    if constexpr (!BF && KT < 4) {
      if (c == KCH - 1) {
#pragma unroll
        for (int st = 0; st < KT; ++st) {
          float wt[NTILE], xt[MT];
#pragma unroll
          for (int nt = 0; nt < NTILE; ++nt)
            wt[nt] = W[(size_t)(nt * 16 + r) * LDW + 16 * c + 4 * st + g];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int src = r + 16 * st;
            const float e0 = __shfl(x[mt][c][0], src), e1 = __shfl(x[mt][c][1], src);
            const float e2 = __shfl(x[mt][c][2], src), e3 = __shfl(x[mt][c][3], src);
            xt[mt] = g == 0 ? e0 : (g == 1 ? e1 : (g == 2 ? e2 : e3));
          }
#pragma unroll
          for (int nt = 0; nt < NTILE; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(wt[nt], xt[mt], acc[mt][nt]);
        }
        continue;
      }
    }
    if constexpr (BF) {
      if (c % 2 == 1) continue;  // taken with chunk c - 1
      const bool pair = c + 1 < KCH;
      const floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
      bf16x8 xb[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) xb[mt] = to_bf16x8(x[mt][c], pair ? x[mt][pair ? c + 1 : c] : z);
#pragma unroll
      for (int nt = 0; nt < NTILE; ++nt) {
        const WT *wp = W + (size_t)(nt * 16 + r) * LDW + 16 * c + 4 * g;
        bf16x8 wb;
        if constexpr (std::is_same<WT, __bf16>::value) {  // staged in BF16 already
          const bf16x4 w0 = *(const bf16x4 *)wp;
          const bf16x4 w1 = pair ? *(const bf16x4 *)(wp + 16) : to_bf16(z);
          wb = __builtin_shufflevector(w0, w1, 0, 1, 2, 3, 4, 5, 6, 7);
        } else {
          const floatx4 w0 = *(const floatx4 *)wp;
          const floatx4 w1 = pair ? *(const floatx4 *)(wp + 16) : z;
          wb = to_bf16x8(w0, w1);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, xb[mt], acc[mt][nt], 0, 0, 0);
      }
      continue;
    }
    floatx4 w[NTILE];
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt)
      w[nt] = *(const floatx4 *)(W + (size_t)(nt * 16 + r) * LDW + 16 * c + 4 * g);
    {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nt = 0; nt < NTILE; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(w[nt][t], x[mt][c][t], acc[mt][nt]);
    }
  }
}

// value of the residual term for output column n: x[n] (identity), x[n mod fin]
// (doubling, where every stored column has n < 2 fin, so n mod fin is one
// conditional subtraction; padding columns read some in-row value and are
// masked by the caller) or 0, read from the wave's LDS copy of its rows.  The
// reads are unconditional (in-row indices) and the mode picks with selects.
__device__ __forceinline__ float res_fwd(const float *rowp, int mode, int fin, int n) {
  const float v = rowp[mode == RES_DOUBLE && n >= fin ? n - fin : n];
  return mode == RES_NONE ? 0.f : v;
}
// Block-shared copies of the small per-column vectors (biases, ws): staged
// once per block, so that no global load sits inside the per-element code.
template <int N>
__device__ __forceinline__ void stage_vec(const float *__restrict__ src, float *dst) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) dst[i] = src[i];
}

struct EmbArgs {
  const float *h1;        // [P][ld0]
  const float *W2t, *b2;  // [ld1][ld0], [ld1]
  const float *W3t, *b3;  // [ld2][ld1], [ld2]
  const float *W2b, *W3b; // [ld0][ld1], [ld1][ld2]  (adjoint operands)
  const float *ws;        // [ld0]
  int n0, n1, n2;         // real widths
  int res2, res3;         // residual rules of layers 2 and 3
  const int *Pptr;
};

// Rows [row0, row0 + 16 MT) of h1 as the B operand of layer 2 (rows past P
// read row 0 and are never stored).
template <int C0, int MT>
__device__ __forceinline__ void load_h1(const float *h1, int row0, int P, int r, int g,
                                        floatx4 (&x0)[MT][C0]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = row0 + mt * 16 + r;
    const int rr = row < P ? row : 0;
#pragma unroll
    for (int c = 0; c < C0; ++c)
      x0[mt][c] = *(const floatx4 *)(h1 + (size_t)rr * (C0 * 16) + 16 * c + 4 * g);
  }
}

// Tiles of the forward as those of the adjoint below: FP32 one 16-row tile
// per wavefront and eight wavefronts per workgroup, BF16 two-tile
// wavefronts, four per workgroup.
constexpr int fwd_tiles(bool bf) { return bf ? 2 : 1; }
constexpr int fwd_waves(bool bf) { return bf ? 4 : 8; }

template <int C0, int C1, int C2, bool BF>
constexpr int emb_fwd_lds_floats();

// W [N][K] into LDS with row stride LDD: FP32, or BF16 (rounded to nearest
// even once here instead of at every use; the same values)
template <int N, int K, int LDD, typename WT>
__device__ __forceinline__ void stage_w(const float *__restrict__ W, WT *dst) {
  for (int idx = threadIdx.x; idx < N * (K / 4); idx += blockDim.x) {
    const int row = idx / (K / 4), c4 = idx % (K / 4);
    const floatx4 v = *(const floatx4 *)(W + (size_t)row * K + 4 * c4);
    if constexpr (std::is_same<WT, __bf16>::value)
      *(bf16x4 *)(dst + row * LDD + 4 * c4) = to_bf16(v);
    else
      *(floatx4 *)(dst + row * LDD + 4 * c4) = v;
  }
}

// LDS row strides (elements) of the staged W2^T [LD1][LD0] and W3^T [LD2][LD1]
// and their size in floats: FP32 rows padded by 4, BF16 rows by 8 (16-byte
// aligned rows either way)
constexpr int w_ld(int k, bool bf) { return bf ? k + 8 : k + 4; }
constexpr int w_floats(int c0, int c1, int c2, bool bf) {
  return bf ? (c1 * 16 * w_ld(c0 * 16, true) + c2 * 16 * w_ld(c1 * 16, true)) / 2
            : c1 * 16 * w_ld(c0 * 16, false) + c2 * 16 * w_ld(c1 * 16, false);
}

template <int C0, int C1, int C2, bool BF>
constexpr int emb_fwd_lds_floats() {
  return fwd_waves(BF) * fwd_tiles(BF) * 16 * (C1 * 16 + 1) + w_floats(C0, C1, C2, BF) +
         C1 * 16 + C2 * 16;
}

// Persistent over row tiles (the grid holds what the device keeps resident,
// two workgroups per CU), with W2^T and W3^T staged in LDS once per
// workgroup (row stride padded by 4 floats).
// T0, T1, T2: MFMA steps of the last depth chunk in contractions over the
// widths n0, n1, n2 (4: the whole chunk; fewer when the real width leaves the
// rest of the chunk zero, FP32 only).
template <int C0, int C1, int C2, bool BF, int T0, int T1, int T2>
__global__ __launch_bounds__(64 * fwd_waves(BF), BF ? 2 : 4) void k_emb_fwd(
    EmbArgs a, float *__restrict__ G0) {
  constexpr int BT = fwd_tiles(BF), BW = fwd_waves(BF);
  constexpr int LD0 = C0 * 16, LD1 = C1 * 16, LD2 = C2 * 16;
  extern __shared__ float esm[];
  float(*xs)[BT * 16][LD1 + 1] = (float(*)[BT * 16][LD1 + 1])esm;  // per wave: h1, then h2 rows
  using WT = typename std::conditional<BF, __bf16, float>::type;
  constexpr int LW2 = w_ld(LD0, BF), LW3 = w_ld(LD1, BF);
  WT *w2s = (WT *)(esm + BW * BT * 16 * (LD1 + 1));  // [LD1][LW2]
  WT *w3s = w2s + LD1 * LW2;                          // [LD2][LW3]
  float *b2s = esm + BW * BT * 16 * (LD1 + 1) + w_floats(C0, C1, C2, BF);
  float *b3s = b2s + LD1;
  const int P = *a.Pptr;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int stride = gridDim.x * BW * 16 * BT;
  int row0 = (blockIdx.x * BW + wave) * 16 * BT;
  stage_vec<LD1>(a.b2, b2s);
  stage_vec<LD2>(a.b3, b3s);
  stage_w<LD1, LD0, LW2>(a.W2t, w2s);
  stage_w<LD2, LD1, LW3>(a.W3t, w3s);
  __syncthreads();
  // the next tile's h1 rows are loaded while the current tile is multiplied
  floatx4 xn[BT][C0];
  if (row0 < P) load_h1<C0>(a.h1, row0, P, lane & 15, lane >> 4, xn);
  for (; row0 < P; row0 += stride) {
    // per-lane indices are taken afresh in every iteration from a value the
    // optimiser cannot see through, so that the addresses derived from them
    // are recomputed here instead of being held in registers across the loop
    int lane_it = lane;
    asm volatile("" : "+v"(lane_it));
    const int r = lane_it & 15, g = lane_it >> 4;
    float(*xw)[LD1 + 1] = xs[wave];
    floatx4 x0[BT][C0];
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int c = 0; c < C0; ++c) x0[mt][c] = xn[mt][c];
    if (row0 + stride < P) load_h1<C0>(a.h1, row0 + stride, P, r, g, xn);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int c = 0; c < C0; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) xw[mt * 16 + r][16 * c + 4 * g + v] = x0[mt][c][v];
    floatx4 acc1[BT][C1];
    layer<C0, C1, BF, T0, LW2>(w2s, r, g, x0, acc1);
    __builtin_amdgcn_wave_barrier();
    floatx4 x1[BT][C1];
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int nt = 0; nt < C1; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const float h =
              tanh_fast(acc1[mt][nt][v] + b2s[n]) + res_fwd(xw[mt * 16 + r], a.res2, a.n0, n);
          x1[mt][nt][v] = n < a.n1 ? h : 0.f;
        }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int nt = 0; nt < C1; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) xw[mt * 16 + r][nt * 16 + 4 * g + v] = x1[mt][nt][v];
    floatx4 acc2[BT][C2];
    layer<C1, C2, BF, T1, LW3>(w3s, r, g, x1, acc2);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mt = 0; mt < BT; ++mt) {
      const int row = row0 + mt * 16 + r;
      if (row >= P) continue;
#pragma unroll
      for (int nt = 0; nt < C2; ++nt) {
        floatx4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const float h =
              tanh_fast(acc2[mt][nt][v] + b3s[n]) + res_fwd(xw[mt * 16 + r], a.res3, a.n1, n);
          o[v] = n < a.n2 ? h : 0.f;
        }
        *(floatx4 *)(G0 + (size_t)row * LD2 + nt * 16 + 4 * g) = o;
      }
    }
  }
}

// acc[mt][nt] = sum_k W[nt*16 + r][k] x[mt][k] with W given by its transpose
// Wt[k][n] (row stride LDT, in LDS): the adjoint products read the forward's
// staged operand.  Same operand values and MFMA order as layer() on W.
template <int KCH, int NTILE, bool BF, int KT, int LDT, int MT, typename WT>
__device__ __forceinline__ void layer_t(const WT *Wt, int r, int g,
                                        const floatx4 (&x)[MT][KCH], floatx4 (&acc)[MT][NTILE]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < KCH; ++c) {
    if constexpr (!BF && KT < 4) {
      if (c == KCH - 1) {
#pragma unroll
        for (int st = 0; st < KT; ++st) {
          float wt[NTILE], xt[MT];
#pragma unroll
          for (int nt = 0; nt < NTILE; ++nt) wt[nt] = Wt[(16 * c + 4 * st + g) * LDT + nt * 16 + r];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int src = r + 16 * st;
            const float e0 = __shfl(x[mt][c][0], src), e1 = __shfl(x[mt][c][1], src);
            const float e2 = __shfl(x[mt][c][2], src), e3 = __shfl(x[mt][c][3], src);
            xt[mt] = g == 0 ? e0 : (g == 1 ? e1 : (g == 2 ? e2 : e3));
          }
#pragma unroll
          for (int nt = 0; nt < NTILE; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(wt[nt], xt[mt], acc[mt][nt]);
        }
        continue;
      }
    }
    if constexpr (BF) {
      if (c % 2 == 1) continue;  // taken with chunk c - 1
      const bool pair = c + 1 < KCH;
      const floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
      bf16x8 xb[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) xb[mt] = to_bf16x8(x[mt][c], pair ? x[mt][pair ? c + 1 : c] : z);
#pragma unroll
      for (int nt = 0; nt < NTILE; ++nt) {
        const WT *wp = Wt + (16 * c + 4 * g) * LDT + nt * 16 + r;
        bf16x8 wb;
        if constexpr (std::is_same<WT, __bf16>::value) {  // staged in BF16 already
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            wb[v] = wp[v * LDT];
            wb[4 + v] = pair ? wp[(16 + v) * LDT] : (__bf16)0.f;
          }
        } else {
          floatx4 w0, w1;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            w0[v] = wp[v * LDT];
            w1[v] = pair ? wp[(16 + v) * LDT] : 0.f;
          }
          wb = to_bf16x8(w0, w1);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, xb[mt], acc[mt][nt], 0, 0, 0);
      }
      continue;
    }
    floatx4 w[NTILE];
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) w[nt][v] = Wt[(16 * c + 4 * g + v) * LDT + nt * 16 + r];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int nt = 0; nt < NTILE; ++nt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(w[nt][t], x[mt][c][t], acc[mt][nt]);
  }
}

// The adjoint's tiles.  FP32: one 16-row tile per wavefront, eight
// wavefronts per workgroup, four wavefronts per SIMD in 128 registers
// (0.54 -> 0.52 ms against two-tile wavefronts at two per SIMD).  BF16 keeps
// two-tile wavefronts, four per workgroup (the one-tile form measured
// 0.28 -> 0.31 ms there).
constexpr int bwd_tiles(bool bf) { return bf ? 2 : 1; }  // 16-row tiles per wavefront
constexpr int bwd_waves(bool bf) { return bf ? 4 : 8; }  // wavefronts per workgroup

template <int C0, int C1, int C2, bool BF>
constexpr int emb_bwd_lds_floats() {
  return bwd_waves(BF) * bwd_tiles(BF) * 16 * (C1 * 16 + 1) + w_floats(C0, C1, C2, BF) +
         C1 * 16 + C2 * 16 + C0 * 16;
}

// Adjoint of layers 2-3 with their forward recomputed, persistent like the
// forward, with W2^T and W3^T staged in LDS (the adjoint products read them
// transposed).  The residual rules of these widths are doubling or none (the
// padded widths differ, so never identity); a doubling residual sends
// d_out[k] + d_out[k + fin] back to input column k, which is formed in the
// wave's LDS rows by storing d_out[k] and then adding d_out[k + fin] in
// place, so a row needs only the input width.
template <int C0, int C1, int C2, bool BF, int T0, int T1, int T2>
__global__ __launch_bounds__(64 * bwd_waves(BF), BF ? 2 : 4) void k_emb_bwd(
    EmbArgs a, const float *__restrict__ dG0, float *__restrict__ gs) {
  constexpr int BT = bwd_tiles(BF), BW = bwd_waves(BF);
  constexpr int LD0 = C0 * 16, LD1 = C1 * 16, LD2 = C2 * 16;
  extern __shared__ float esm[];
  float(*xs)[BT * 16][LD1 + 1] = (float(*)[BT * 16][LD1 + 1])esm;  // per wave: h1, then folds
  using WT = typename std::conditional<BF, __bf16, float>::type;
  constexpr int LW2 = w_ld(LD0, BF), LW3 = w_ld(LD1, BF);
  WT *w2s = (WT *)(esm + BW * BT * 16 * (LD1 + 1));  // [LD1][LW2]
  WT *w3s = w2s + LD1 * LW2;                          // [LD2][LW3]
  float *b2s = esm + BW * BT * 16 * (LD1 + 1) + w_floats(C0, C1, C2, BF);
  float *b3s = b2s + LD1;
  float *wss = b3s + LD2;
  const int P = *a.Pptr;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int stride = gridDim.x * BW * 16 * BT;
  stage_vec<LD1>(a.b2, b2s);
  stage_vec<LD2>(a.b3, b3s);
  stage_vec<LD0>(a.ws, wss);
  stage_w<LD1, LD0, LW2>(a.W2t, w2s);
  stage_w<LD2, LD1, LW3>(a.W3t, w3s);
  __syncthreads();
  // per-lane indices taken afresh in every iteration, as in the forward
  for (int row0 = (blockIdx.x * BW + wave) * 16 * BT; row0 < P; row0 += stride) {
  int lane_it = lane;
  asm volatile("" : "+v"(lane_it));
  const int r = lane_it & 15, g = lane_it >> 4;
  float(*xw)[LD1 + 1] = xs[wave];
  __builtin_amdgcn_wave_barrier();
  // ---- recompute the forward
  floatx4 x0[BT][C0];
  load_h1<C0>(a.h1, row0, P, r, g, x0);
#pragma unroll
  for (int mt = 0; mt < BT; ++mt)
#pragma unroll
    for (int c = 0; c < C0; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) xw[mt * 16 + r][16 * c + 4 * g + v] = x0[mt][c][v];
  floatx4 t1[BT][C1], x1[BT][C1];
  {
    floatx4 acc1[BT][C1];
    layer<C0, C1, BF, T0, LW2>(w2s, r, g, x0, acc1);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int nt = 0; nt < C1; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const float t = tanh_fast(acc1[mt][nt][v] + b2s[n]);
          const float h = t + res_fwd(xw[mt * 16 + r], a.res2, a.n0, n);
          t1[mt][nt][v] = n < a.n1 ? t : 0.f;
          x1[mt][nt][v] = n < a.n1 ? h : 0.f;
        }
  }
  floatx4 d2[BT][C2];  // tanh output of layer 3, then dE/du3
  {
    floatx4 acc2[BT][C2];
    layer<C1, C2, BF, T1, LW3>(w3s, r, g, x1, acc2);
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int nt = 0; nt < C2; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const float t = tanh_fast(acc2[mt][nt][v] + b3s[n]);
          d2[mt][nt][v] = n < a.n2 ? t : 0.f;
        }
  }
  // ---- adjoint: du3 = dG0 (1 - t3^2); the wave's rows get dG0[k] + dG0[k + n1]
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int mt = 0; mt < BT; ++mt) {
    const int row = row0 + mt * 16 + r;
    const int rr = row < P ? row : 0;
    floatx4 gv[C2];  // all loads of the tile row before any use
#pragma unroll
    for (int nt = 0; nt < C2; ++nt)
      gv[nt] = *(const floatx4 *)(dG0 + (size_t)rr * LD2 + nt * 16 + 4 * g);
#pragma unroll
    for (int nt = 0; nt < C2; ++nt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (nt < C1) xw[mt * 16 + r][nt * 16 + 4 * g + v] = gv[nt][v];
        const float t = d2[mt][nt][v];
        d2[mt][nt][v] = gv[nt][v] * (1.0f - t * t);
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (a.res3 == RES_DOUBLE) {
#pragma unroll
      for (int nt = 0; nt < C2; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          if (n >= a.n1 && n < a.n2) xw[mt * 16 + r][n - a.n1] += gv[nt][v];
        }
    }
  }
  __builtin_amdgcn_wave_barrier();
  // dh2 = du3 W3^T + res^T(dG0) ; du2 = dh2 (1 - t2^2)
  floatx4 du2[BT][C1];
  {
    floatx4 acc[BT][C1];
    layer_t<C2, C1, BF, T2, LW3>(w3s, r, g, d2, acc);
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int nt = 0; nt < C1; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = nt * 16 + 4 * g + v;
          const float res = a.res3 == RES_NONE ? 0.f : xw[mt * 16 + r][k];
          const float dd = acc[mt][nt][v] + res;
          const float d = k < a.n1 ? dd : 0.f;
          acc[mt][nt][v] = d;  // dh2
          const float t = t1[mt][nt][v];
          du2[mt][nt][v] = d * (1.0f - t * t);
        }
    // the wave's rows get dh2[k] + dh2[k + n0]
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mt = 0; mt < BT; ++mt)
#pragma unroll
      for (int nt = 0; nt < C0; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) xw[mt * 16 + r][nt * 16 + 4 * g + v] = acc[mt][nt][v];
    __builtin_amdgcn_wave_barrier();
    if (a.res2 == RES_DOUBLE) {
#pragma unroll
      for (int mt = 0; mt < BT; ++mt)
#pragma unroll
        for (int nt = 0; nt < C1; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = nt * 16 + 4 * g + v;
            if (n >= a.n0 && n < a.n1) xw[mt * 16 + r][n - a.n0] += acc[mt][nt][v];
          }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // dh1 = du2 W2^T + res^T(dh2) ; du1 = dh1 (1 - h1^2) ; gs = du1 . ws
  floatx4 acc0[BT][C0];
  layer_t<C1, C0, BF, T1, LW2>(w2s, r, g, du2, acc0);
  // one-tile wavefronts read their h1 rows again (from L2) rather than hold
  // them in registers through the adjoint, which spilled at 128 registers
  if constexpr (BT == 1) load_h1<C0>(a.h1, row0, P, r, g, x0);
#pragma unroll
  for (int mt = 0; mt < BT; ++mt) {
    float s = 0.f;
#pragma unroll
    for (int nt = 0; nt < C0; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = nt * 16 + 4 * g + v;
        const float res = a.res2 == RES_NONE ? 0.f : xw[mt * 16 + r][k];
        const float d = acc0[mt][nt][v] + res;
        const float h = x0[mt][nt][v];
        const float term = d * (1.0f - h * h) * wss[k];
        s += k < a.n0 ? term : 0.f;
      }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    const int row = row0 + mt * 16 + r;
    if (g == 0 && row < P) gs[row] = s;
  }
  }
}

// Instantiated widths (padded to 16): the benchmark model's 32/64/112
// (25/50/100) and the distilled student's 16/32/64.
bool is_student_widths(int ld0, int ld1, int ld2) { return ld0 == 16 && ld1 == 32 && ld2 == 64; }

}  // namespace

bool emb_fused_supported(int ld0, int ld1, int ld2) {
  return (ld0 == 32 && ld1 == 64 && ld2 == 112) || is_student_widths(ld0, ld1, ld2);
}

namespace {

// Blocks of kernel k that the device holds at once (the persistent grid).
template <class K>
unsigned resident_blocks(K k, size_t lds = 0, int threads = 256) {
  int nb = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, lds) != hipSuccess || nb <= 0)
    nb = 2;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return (unsigned)(nb * cus);
}

template <int C0, int C1, int C2, bool BF, int T0 = 4, int T1 = 4, int T2 = 4>
void emb_fwd_grid(const EmbArgs &a, long rows, float *G0, hipStream_t s) {
  constexpr size_t lds = sizeof(float) * emb_fwd_lds_floats<C0, C1, C2, BF>();
  constexpr int threads = 64 * fwd_waves(BF);
  constexpr long per_block = 16L * fwd_tiles(BF) * fwd_waves(BF);  // rows per block and round
  const long tiles = (rows + per_block - 1) / per_block;
  static unsigned cap = 0;
  if (cap == 0) {
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void *)k_emb_fwd<C0, C1, C2, BF, T0, T1, T2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    cap = resident_blocks(k_emb_fwd<C0, C1, C2, BF, T0, T1, T2>, lds, threads);
  }
  const unsigned blocks = (unsigned)(tiles < (long)cap ? tiles : (long)cap);
  hipLaunchKernelGGL((k_emb_fwd<C0, C1, C2, BF, T0, T1, T2>), dim3(blocks), dim3(threads), lds,
                     s, a, G0);
}

template <int C0, int C1, int C2, bool BF, int T0 = 4, int T1 = 4, int T2 = 4>
void emb_bwd_grid(const EmbArgs &a, long rows, const float *dG0, float *gs, hipStream_t s) {
  constexpr size_t lds = sizeof(float) * emb_bwd_lds_floats<C0, C1, C2, BF>();
  constexpr int threads = 64 * bwd_waves(BF);
  constexpr long per_block = 16L * bwd_tiles(BF) * bwd_waves(BF);  // rows per block and round
  const long tiles = (rows + per_block - 1) / per_block;
  static unsigned cap = 0;
  if (cap == 0) {
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void *)k_emb_bwd<C0, C1, C2, BF, T0, T1, T2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    cap = resident_blocks(k_emb_bwd<C0, C1, C2, BF, T0, T1, T2>, lds, threads);
  }
  const unsigned blocks = (unsigned)(tiles < (long)cap ? tiles : (long)cap);
  hipLaunchKernelGGL((k_emb_bwd<C0, C1, C2, BF, T0, T1, T2>), dim3(blocks), dim3(threads), lds,
                     s, a, dG0, gs);
}

// MFMA steps that the last 16-wide depth chunk of a contraction over real
// width n needs (the chunk holds n - 16 (pad16(n) / 16 - 1) real columns).
int tail_steps(int n) { return (n - (pad16(n) - 16) + 3) / 4; }

// The benchmark model's widths 25 / 50 / 100 in FP32: 3, 1 and 1 steps.
bool short_tails(const EmbLaunch &e) {
  return !e.bf16 && tail_steps(e.n0) == 3 && tail_steps(e.n1) == 1 && tail_steps(e.n2) == 1;
}

}  // namespace

void launch_emb_fwd(const EmbLaunch &e, float *G0, hipStream_t s) {
  EmbArgs a{e.h1, e.W2t, e.b2, e.W3t, e.b3, e.W2b, e.W3b, e.ws, e.n0, e.n1, e.n2, e.res2, e.res3,
            e.Pptr};
  const long rows = e.Pmax;
  if (rows <= 0) return;
  const bool st = is_student_widths(pad16(e.n0), pad16(e.n1), pad16(e.n2));
  if (st && e.bf16) emb_fwd_grid<1, 2, 4, true>(a, rows, G0, s);
  else if (st) emb_fwd_grid<1, 2, 4, false>(a, rows, G0, s);
  else if (e.bf16) emb_fwd_grid<2, 4, 7, true>(a, rows, G0, s);
  else if (short_tails(e)) emb_fwd_grid<2, 4, 7, false, 3, 1, 1>(a, rows, G0, s);
  else emb_fwd_grid<2, 4, 7, false>(a, rows, G0, s);
}

void launch_emb_bwd(const EmbLaunch &e, const float *dG0, float *gs, hipStream_t s) {
  EmbArgs a{e.h1, e.W2t, e.b2, e.W3t, e.b3, e.W2b, e.W3b, e.ws, e.n0, e.n1, e.n2, e.res2, e.res3,
            e.Pptr};
  const long rows = e.Pmax;
  if (rows <= 0) return;
  const bool st = is_student_widths(pad16(e.n0), pad16(e.n1), pad16(e.n2));
  if (st && e.bf16) emb_bwd_grid<1, 2, 4, true>(a, rows, dG0, gs, s);
  else if (st) emb_bwd_grid<1, 2, 4, false>(a, rows, dG0, gs, s);
  else if (e.bf16) emb_bwd_grid<2, 4, 7, true>(a, rows, dG0, gs, s);
  else if (short_tails(e)) emb_bwd_grid<2, 4, 7, false, 3, 1, 1>(a, rows, dG0, gs, s);
  else emb_bwd_grid<2, 4, 7, false>(a, rows, dG0, gs, s);
}

}  // namespace dpa1
