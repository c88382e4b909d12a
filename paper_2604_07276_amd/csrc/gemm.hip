// Row-batched FP32 GEMMs on the CDNA matrix cores, with fused epilogues.
//
// Every multilayer-perceptron layer of the model (the embedding net, the
// attention input/output projections and the fitting net, Sec. II-B) and its
// input-gradient adjoint is a product Y[M x N] = X[M x K] W[K x N] with a
// small weight matrix shared by all rows (neighbour pairs or centres).
//
// Tiling: one wavefront owns 16*MT rows and NT tiles of 16 output columns.
// The kernel computes the transposed product Y^T = W^T X^T with
// v_mfma_f32_16x16x4_f32 so that the accumulator layout gives each lane four
// consecutive output columns of one row: lane l holds row (l % 16) and
// columns 4*(l / 16) + {0..3} of every 16x16 tile, which makes the epilogue
// stores 16-byte vector stores and the per-row reductions of the layer norm
// a register sum plus two cross-lane steps.  Both operands are read as
// 16-byte vectors along k straight from global memory (W is stored
// transposed, Wt[n][k]); the k index of a 16-wide chunk is permuted
// identically on both operands, which leaves the contraction unchanged.
#include "dpa1_internal.h"
#include "ln_res.h"

namespace dpa1 {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 precision mode: gfx950's v_mfma_f32_16x16x32_bf16 takes two 16-wide
// k chunks at once.  Lane l holds, for row l % 16, the four consecutive
// values k = 4 (l / 16) + 0..3 of each chunk (the values the FP32 path feeds
// to four 16x16x4 steps per chunk); its eight operand slots are the first
// chunk's four followed by the second chunk's four, on both operands alike,
// which gives exactly the sum of two v_mfma_f32_16x16x16_bf16 steps (checked
// on the hardware).  A lone last chunk is paired with zero weights.
// Operands are rounded to BF16 (nearest even) in registers, accumulation
// stays FP32.
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

// X operand storage: BF selects the matrix-core operand precision (0 FP32,
// 1 BF16 operands from an FP32 X, 2 BF16 operands from an X stored in BF16).
// p points at element 0 of the lane's run of four in the X storage type.
template <int BF>
__device__ __forceinline__ const float *x_at(const float *X, size_t elem) {
  if constexpr (BF == 2) return (const float *)((const __bf16 *)X + elem);
  else return X + elem;
}
template <int BF>
__device__ __forceinline__ floatx4 ldx4(const float *p, int k) {
  if constexpr (BF == 2)
    return __builtin_convertvector(*(const bf16x4 *)((const __bf16 *)p + k), floatx4);
  else
    return *(const floatx4 *)(p + k);
}

__device__ __forceinline__ float row_sum16(float v) {
  // sum over the four lane groups that share (lane % 16)
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

template <class Epi, int NT>
__device__ void stage_cols(const Epi &e, int nt0, int npad, float *cs);

template <int MT, int NT, class Epi, int BF>
__global__ __launch_bounds__(256, MT >= 4 ? 2 : 3) void k_gemm(GemmArgs a, Epi epi) {
  __shared__ float cs[Epi::kCols * NT * 16];
  // The block's W^T rows of one 16-deep k chunk, double-buffered: the four
  // wavefronts share each chunk instead of each reading it from L2.
  // Used by the BF16 instances and the 16-row (per-centre) tiles; the FP32
  // 64-row tiles keep per-wavefront W streams (see the k loop).
  constexpr bool kShareW = BF != 0 || MT < 4;
  // k depth of one staged chunk: 32 in BF16 (one 16x16x32 step) and for the
  // FP32 16-row tiles (the long-k fitting products: two 16-deep steps per
  // barrier, the next chunk's loads twice as far ahead); 16 for FP32 32-row
  // tiles (whose registers a 32-deep chunk would spill)
  constexpr int KC = (BF != 0 || MT == 1) ? 32 : 16;
  constexpr int H = KC / 16;        // 16-deep steps per chunk
  constexpr int kWS = KC + 4;       // LDS row stride
  __shared__ float wsh[kShareW ? 2 : 1][kShareW ? NT * 16 : 1][kWS];
  const int M = a.Mptr ? *a.Mptr : a.Mmax;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int nt0 = blockIdx.y * NT;
  stage_cols<Epi, NT>(epi, nt0, a.Npad, cs);
  __syncthreads();
  const int ntt = a.Npad / 16;
  // k range of this workgroup: all of K, or with split k (shared-W paths
  // only, kslice a multiple of the chunk depth) slice blockIdx.z
  const int kbeg = a.kslice ? (int)blockIdx.z * a.kslice : 0;
  const int kend = a.kslice ? min(a.K, kbeg + a.kslice) : a.K;
  // W staging: thread tid moves float4 q = tid + 256 j of the chunk, row
  // q / QPR of the block's W^T rows, k quad q % QPR (column tiles past the
  // last one stage a duplicate of tile 0; their outputs are never stored).
  // A 32-deep chunk that runs past K (a multiple of 16) stages zeros for its
  // second half.
  constexpr int QPR = KC / 4;
  constexpr int NQ = NT * 16 * QPR;
  constexpr int JW = (NQ + 255) / 256;
  const float *wsrc[JW];
#pragma unroll
  for (int j = 0; j < JW; ++j) {
    const int q = tid + 256 * j < NQ ? tid + 256 * j : 0;
    const int n = q / QPR;
    const int tile = nt0 + n / 16 < ntt ? nt0 + n / 16 : 0;
    wsrc[j] = a.Wt + (size_t)(tile * 16 + n % 16) * a.K + 4 * (q % QPR);
  }
  // persistent over row tiles: the grid is sized to the resident capacity
  // (launch gaps and the tail of short-lived waves otherwise cost ~40%).
  // Every wavefront of a block runs the same iterations (the block-level
  // barriers of the k loop need all four): a wavefront whose rows are all
  // past M computes on row 0 and stores nothing.
  for (int blk0 = blockIdx.x * 64 * MT; blk0 < M; blk0 += gridDim.x * 64 * MT) {
  const int row0 = blk0 + wave * 16 * MT;
  // per-lane offsets are recomputed in every iteration from an index the
  // optimiser cannot see through, instead of being held across the loop
  int lane_it = lane;
  asm volatile("" : "+v"(lane_it));
  const int r = lane_it & 15;
  const int g = lane_it >> 4;

  floatx4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};

  const float *xrow[MT];
  bool xok[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = row0 + mt * 16 + r;
    xok[mt] = row < M;  // rows past M read row 0 and are never stored
    xrow[mt] = x_at<BF>(a.X, (size_t)(xok[mt] ? row : 0) * a.ldx + 4 * g);
  }
  if constexpr (kShareW) {
    float4 wst[JW];
    auto wload = [&](int k) {
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        // a quad of the second half past K (16-deep tail) reads the first
        // half's address and stages zeros
        const int q = tid + 256 * j < NQ ? tid + 256 * j : 0;  // as in wsrc
        const bool ok = KC == 16 || k + 4 * (q % QPR) < kend;
        const float4 v = *(const float4 *)(wsrc[j] + (ok ? k : k - 16));
        wst[j] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    auto wstore = [&](int b) {
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const int q = tid + 256 * j;
        if (NQ % 256 == 0 || q < NQ) *(float4 *)&wsh[b][q / QPR][4 * (q % QPR)] = wst[j];
      }
    };
  if constexpr (BF != 0) {
    // BF16: 32-deep chunks, one 16x16x32 step per tile pair.  The next
    // chunk's X quads (k0 + 4g and k0 + 16 + 4g; past K the second re-reads
    // the first, which meets zero weights) are loaded in FP32 while the
    // current chunk, already rounded to BF16, is multiplied; each W tile is
    // read from LDS and rounded just before its MFMAs.
    floatx4 xn[MT][2];
    bf16x8 xb[MT];
    auto xload = [&](int k0) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        xn[mt][0] = ldx4<BF>(xrow[mt], k0);
        xn[mt][1] = ldx4<BF>(xrow[mt], k0 + 16 < kend ? k0 + 16 : k0);
      }
    };
    wload(kbeg);
    xload(kbeg);
    wstore(0);
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) xb[mt] = to_bf16x8(xn[mt][0], xn[mt][1]);
    int b = 0;
#pragma unroll 1
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
      const bool more = k0 + KC < kend;  // uniform
      if (more) {
        wload(k0 + KC);
        xload(k0 + KC);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const floatx4 w0 = *(const floatx4 *)&wsh[b][nt * 16 + r][4 * g];
        const floatx4 w1 = *(const floatx4 *)&wsh[b][nt * 16 + r][16 + 4 * g];
        const bf16x8 wb = to_bf16x8(w0, w1);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_bf16x2(wb, xb[mt], acc[mt][nt]);
      }
      if (more) wstore(b ^ 1);
      __syncthreads();  // chunk k0 + KC staged; buffer b free again
      b ^= 1;
      if (more) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) xb[mt] = to_bf16x8(xn[mt][0], xn[mt][1]);
      }
    }
  } else {

    // Double-buffered k loop: the operands of chunk k0 + KC (the block's W
    // rows, the wavefront's X rows) are loaded while chunk k0 is multiplied
    // as H 16-deep steps (with H = 2 a second half past K, K being a
    // multiple of 16, re-reads the first half of X and meets zero weights:
    // its MFMAs add zeros); the MFMAs of one step go to independent
    // accumulators back to back.
    floatx4 xv[MT][H], xn[MT][H];
    auto xload = [&](int k0, floatx4 (&x)[MT][H]) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int h = 0; h < H; ++h)
          x[mt][h] = ldx4<BF>(xrow[mt], k0 + 16 * h < kend ? k0 + 16 * h : k0);
    };
    wload(kbeg);
    xload(kbeg, xv);
    wstore(0);
    __syncthreads();
    int b = 0;
#pragma unroll 1
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
      const bool more = k0 + KC < kend;  // uniform
      if (more) {
        wload(k0 + KC);
        xload(k0 + KC, xn);
      }
#pragma unroll
      for (int h = 0; h < H; ++h) {
        floatx4 wv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          wv[nt] = *(const floatx4 *)&wsh[b][nt * 16 + r][16 * h + 4 * g];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][nt] = mfma4(wv[nt][t], xv[mt][h][t], acc[mt][nt]);
      }
      if (more) wstore(b ^ 1);
      __syncthreads();  // chunk k0 + KC staged; buffer b free again
      b ^= 1;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int h = 0; h < H; ++h) xv[mt][h] = xn[mt][h];
    }
  }
  } else {
    // FP32 64-row tiles: each wavefront streams its own W rows from L2 (the
    // per-chunk block barrier of the shared staging costs these long-K
    // products more than the L2 reads it saves)
    const float *wrow[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int tile = nt0 + nt < ntt ? nt0 + nt : 0;
      wrow[nt] = a.Wt + (size_t)(tile * 16 + r) * a.K + 4 * g;
    }
    floatx4 xv[MT], wv[NT], xn[MT], wn[NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) xv[mt] = ldx4<BF>(xrow[mt], 0);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) wv[nt] = *(const floatx4 *)(wrow[nt]);
#pragma unroll 1
    for (int k0 = 0; k0 < a.K; k0 += 16) {
      const int kn = k0 + 16 < a.K ? k0 + 16 : k0;  // last chunk reloads itself (unused)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) xn[mt] = ldx4<BF>(xrow[mt], kn);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) wn[nt] = *(const floatx4 *)(wrow[nt] + kn);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(wv[nt][t], xv[mt][t], acc[mt][nt]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) xv[mt] = xn[mt];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) wv[nt] = wn[nt];
    }
  }
  epi.template apply<MT, NT>(acc, row0, nt0, ntt, lane, M, cs);
  }
}

// Persistent variant for the large pair-batched products whose weight tile
// fits in LDS (K = KCH*16 <= 128): each workgroup stages its W^T column
// block [NT*16][K] in LDS once and then walks over row tiles (4 waves x
// 16*MT rows), so weights are read from L2 once per workgroup instead of once
// per wavefront.  A wavefront holds the whole K extent of its rows in
// registers and loads the rows of its next tile while it multiplies the
// current one, so the HBM latency of the activations is paid once per
// launch rather than once per tile.  gridDim.x is a multiple of 8 so that
// the column blocks of one row tile are dispatched to the same XCD (shared
// L2 for the activations).
// KT = 1 (FP32 only): X holds data only in the first four columns of its last
// 16-wide chunk (zeros past them).  That chunk then takes one MFMA step in
// which lane group g carries depth 16 (KCH - 1) + g on both operands, instead
// of four steps over mostly zero columns; the lane loads that one value.
template <int MT, int KCH, int BF, int KT>
__device__ __forceinline__ void load_x_tile(const GemmArgs &a, int row0, int M, int r, int g,
                                            floatx4 (&x)[MT][KCH]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = row0 + mt * 16 + r;
    const float *xp = x_at<BF>(a.X, (size_t)(row < M ? row : 0) * a.ldx + 4 * g);
#pragma unroll
    for (int c = 0; c < KCH; ++c) {
      if (KT == 1 && c == KCH - 1)
        x[mt][c][0] = xp[16 * c - 3 * g];  // column 16 c + g of the row
      else
        x[mt][c] = ldx4<BF>(xp, 16 * c);
    }
  }
}

template <int MT, int NT, int KCH, class Epi, int BF, int KT>
__global__ __launch_bounds__(256, 2) void k_gemm_lds(GemmArgs a, Epi epi) {
  constexpr int K = KCH * 16;
  constexpr int LDW = K + 4;
  extern __shared__ float wsm[];  // [NT * 16][LDW]
  const int M = a.Mptr ? *a.Mptr : a.Mmax;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int nt0 = blockIdx.y * NT;
  const int ntt = a.Npad / 16;
  const int r = lane & 15;
  const int g = lane >> 4;
  for (int idx = threadIdx.x; idx < NT * 16 * KCH * 4; idx += blockDim.x) {
    const int row = idx / (KCH * 4), c4 = idx % (KCH * 4);
    const int n = nt0 * 16 + row;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (n < a.Npad) v = *(const float4 *)(a.Wt + (size_t)n * a.K + 4 * c4);
    *(float4 *)(wsm + row * LDW + 4 * c4) = v;
  }
  float *cs = wsm + NT * 16 * LDW;  // [Epi::kCols][NT * 16]
  stage_cols<Epi, NT>(epi, nt0, a.Npad, cs);
  __syncthreads();
  const float *wl = wsm + r * LDW + 4 * g;
  const int stride = gridDim.x * 64 * MT;  // rows between a wave's consecutive tiles
  int row0 = (blockIdx.x * 4 + wave) * 16 * MT;
  if constexpr (BF != 0) {
    // BF16: chunks 2p and 2p + 1 in one 16x16x32 step (a lone last chunk is
    // paired with zeros on both operands).  The current tile is held as BF16
    // chunk pairs; the next one arrives in FP32 and is rounded once.
    constexpr int KP = (KCH + 1) / 2;
    floatx4 xn[MT][KCH];
    bf16x8 xc[MT][KP];
    auto to_pairs = [&]() {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int p = 0; p < KP; ++p)
          xc[mt][p] = to_bf16x8(xn[mt][2 * p],
                                2 * p + 1 < KCH ? xn[mt][2 * p + 1] : floatx4{0.f, 0.f, 0.f, 0.f});
    };
    if (row0 < M) {
      load_x_tile<MT, KCH, BF, KT>(a, row0, M, r, g, xn);
      to_pairs();
    }
    for (; row0 < M; row0 += stride) {
      const bool next = row0 + stride < M;
      if constexpr (Epi::kLds == 1)
        if (next) load_x_tile<MT, KCH, BF, KT>(a, row0 + stride, M, r, g, xn);
      floatx4 acc[MT][NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int p = 0; p < KP; ++p) {
        bf16x8 wb[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const floatx4 w0 = *(const floatx4 *)(wl + nt * 16 * LDW + 32 * p);
          const floatx4 w1 = 2 * p + 1 < KCH ? *(const floatx4 *)(wl + nt * 16 * LDW + 32 * p + 16)
                                             : floatx4{0.f, 0.f, 0.f, 0.f};
          wb[nt] = to_bf16x8(w0, w1);
        }
        __builtin_amdgcn_sched_barrier(0);  // one chunk pair of weights live at a time
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_bf16x2(wb[nt], xc[mt][p], acc[mt][nt]);
      }
      if constexpr (Epi::kLds == 2)
        if (next) load_x_tile<MT, KCH, BF, KT>(a, row0 + stride, M, r, g, xn);
      epi.template apply<MT, NT>(acc, row0, nt0, ntt, lane, M, cs);
      if (next) to_pairs();
    }
    return;
  }
  floatx4 xr[MT][KCH], xn[MT][KCH];
  if (row0 < M) load_x_tile<MT, KCH, BF, KT>(a, row0, M, r, g, xr);
  for (; row0 < M; row0 += stride) {
    // the layer-norm epilogue holds more registers: its prefetch waits until
    // the current tile's activations are dead
    if constexpr (Epi::kLds == 1)
      if (row0 + stride < M) load_x_tile<MT, KCH, BF, KT>(a, row0 + stride, M, r, g, xn);
    floatx4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KCH; ++c) {
      if constexpr (KT == 1 && BF == 0) {
        if (c == KCH - 1) {
          // one step: depth 16 c + g on both operands (W from LDS at that depth)
          const float *wt = wsm + r * LDW + 16 * c + g;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const float wv = wt[nt * 16 * LDW];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(wv, xr[mt][c][0], acc[mt][nt]);
          }
          continue;
        }
      }
      floatx4 w[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) w[nt] = *(const floatx4 *)(wl + nt * 16 * LDW + 16 * c);
      __builtin_amdgcn_sched_barrier(0);  // one chunk of weights live at a time
      {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][nt] = mfma4(w[nt][t], xr[mt][c][t], acc[mt][nt]);
      }
    }
    if constexpr (Epi::kLds == 2)
      if (row0 + stride < M) load_x_tile<MT, KCH, BF, KT>(a, row0 + stride, M, r, g, xn);
    epi.template apply<MT, NT>(acc, row0, nt0, ntt, lane, M, cs);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int c = 0; c < KCH; ++c) xr[mt][c] = xn[mt][c];
  }
}

// Resident-weight variant for the long-K FP32 adjoint of the QKV projection
// (K = KCH*16 = 384 rows of W, Nreal <= NT*16 output columns): the whole
// W^T[Nreal][K] block lives in LDS for the launch (one 8-wavefront workgroup
// per CU), so the k loop has no barrier and reads no weights from L2.  Each
// wavefront walks its own 64-row tiles independently and streams X through
// a ring of three 16-deep chunks, two chunks ahead of the one it multiplies;
// the ring runs on across tile boundaries, so the next tile's first chunks
// arrive during the current tile's last ones and its epilogue.  Output
// columns past Nreal read a clamped W row; the epilogue zeroes them.
template <int MT, int NT, int KCH, class Epi>
__global__ __launch_bounds__(512, 1) void k_gemm_wres(GemmArgs a, Epi epi) {
  static_assert(KCH % 3 == 0, "the chunk ring is unrolled by three");
  constexpr int K = KCH * 16;
  constexpr int LDW = K + 4;
  extern __shared__ float wsm[];  // [Nreal][LDW], then cs
  const int M = a.Mptr ? *a.Mptr : a.Mmax;
  const int nreal = a.Nreal;
  for (int idx = threadIdx.x; idx < nreal * (K / 4); idx += blockDim.x) {
    const int n = idx / (K / 4), c4 = idx % (K / 4);
    *(float4 *)(wsm + n * LDW + 4 * c4) = *(const float4 *)(a.Wt + (size_t)n * a.K + 4 * c4);
  }
  float *cs = wsm + nreal * LDW;  // [Epi::kCols][NT * 16]
  stage_cols<Epi, NT>(epi, 0, a.Npad, cs);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int ntt = a.Npad / 16;
  // wave-major tile order: the tiles left over after the last full round
  // land on different CUs (1.21 -> 1.16 ms against the block-major order)
  const int stride = gridDim.x * 8 * 16 * MT;  // rows between a wave's consecutive tiles
  int row0 = (wave * gridDim.x + blockIdx.x) * 16 * MT;
  if (row0 >= M) return;  // no barrier follows
  int lane_it = lane;
  asm volatile("" : "+v"(lane_it));
  const int r = lane_it & 15;
  const int g = lane_it >> 4;
  const float *wl[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = nt * 16 + r < nreal ? nt * 16 + r : nreal - 1;
    wl[nt] = wsm + n * LDW + 4 * g;
  }
  auto rows_of = [&](int base, const float *(&xp)[MT]) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = base + mt * 16 + r;
      xp[mt] = a.X + (size_t)(row < M ? row : 0) * a.ldx + 4 * g;
    }
  };
  const float *xc[MT], *xn[MT];
  rows_of(row0, xc);
  rows_of(row0 + stride, xn);
  floatx4 xb[3][MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    xb[0][mt] = *(const floatx4 *)(xc[mt]);
    xb[1][mt] = *(const floatx4 *)(xc[mt] + 16);
  }
  for (; row0 < M; row0 += stride) {
    floatx4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int c = 0; c < KCH; c += 3) {
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        // chunk c + u sits in slot u; chunk c + u + 2 (of this tile, or of
        // the next one past the last chunk) goes into the slot freed by the
        // previous step
        const int cp = c + u + 2;
        const bool here = cp < KCH;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          xb[(u + 2) % 3][mt] = *(const floatx4 *)(here ? xc[mt] + 16 * cp : xn[mt] + 16 * (cp - KCH));
        floatx4 w[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) w[nt] = *(const floatx4 *)(wl[nt] + 16 * (c + u));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(w[nt][t], xb[u][mt][t], acc[mt][nt]);
      }
    }
    epi.template apply<MT, NT>(acc, row0, 0, ntt, lane, M, cs);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) xc[mt] = xn[mt];
    rows_of(row0 + 2 * stride, xn);
  }
}

// Product with several column blocks (the QKV projection: 24 tiles)
// whose data fills only the first four columns of its last k chunk: the
// whole W^T block (CB x NT x 16 rows of 16 (KCH - 1) + 4 staged columns,
// 160 KB for 384 x 100) is resident in LDS for the launch, one
// eight-wavefront workgroup per CU.  Each wavefront holds a 32-row tile of X
// in registers and produces its CB column blocks one after the other, so X
// is read from memory once instead of once per column block; the next row
// tile is loaded while the current one is multiplied.  Tiles are taken in
// wave-major order (the last round's tiles land on different CUs).
// BF = 1: BF16 operands (X still FP32 in memory), chunks 2p and 2p + 1 in
// one 16x16x32 step, the lone last chunk (four real columns, held by lane
// group 0 only) paired with zeros.
template <int NT, int CB, int KCH, class Epi, int BF>
__global__ __launch_bounds__(512, 1) void k_gemm_cols(GemmArgs a, Epi epi) {
  static_assert(Epi::kCols == 1, "one staged column vector");
  constexpr int MT = 2;
  constexpr int KS = 16 * (KCH - 1) + 4;  // staged depth
  constexpr int LDW = KS + 4;
  constexpr int NC = CB * NT * 16;  // staged output columns
  extern __shared__ float wsm[];    // [NC][LDW], then the column vector [NC]
  const int M = a.Mptr ? *a.Mptr : a.Mmax;
  for (int idx = threadIdx.x; idx < NC * (KS / 4); idx += blockDim.x) {
    const int row = idx / (KS / 4), c4 = idx % (KS / 4);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < a.Npad) v = *(const float4 *)(a.Wt + (size_t)row * a.K + 4 * c4);
    *(float4 *)(wsm + row * LDW + 4 * c4) = v;
  }
  float *cs = wsm + NC * LDW;
  stage_cols<Epi, CB * NT>(epi, 0, a.Npad, cs);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int g = lane >> 4;
  const int ntt = a.Npad / 16;
  const int stride = gridDim.x * 8 * 16 * MT;  // rows between a wave's consecutive tiles
  int row0 = (wave * gridDim.x + blockIdx.x) * 16 * MT;
  if constexpr (BF != 0) {
    constexpr int KP = (KCH + 1) / 2;
    static_assert(KCH % 2 == 1, "the last chunk is the lone one");
    floatx4 xn[MT][KCH];
    bf16x8 xc[MT][KP];
    const floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
    auto to_pairs = [&]() {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int p = 0; p < KP; ++p)
          xc[mt][p] = to_bf16x8(xn[mt][2 * p], 2 * p + 1 < KCH ? xn[mt][2 * p + 1] : z);
    };
    if (row0 < M) {
      load_x_tile<MT, KCH, 1, 4>(a, row0, M, r, g, xn);
      to_pairs();
    }
    for (; row0 < M; row0 += stride) {
      const bool next = row0 + stride < M;
      if (next) load_x_tile<MT, KCH, 1, 4>(a, row0 + stride, M, r, g, xn);
#pragma unroll 1
      for (int cb = 0; cb < CB; ++cb) {
        floatx4 acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = z;
        const float *wb = wsm + (cb * NT * 16 + r) * LDW + 4 * g;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
          bf16x8 w[NT];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const float *wp = wb + nt * 16 * LDW + 32 * p;
            floatx4 w0, w1;
            if (2 * p + 1 < KCH) {
              w0 = *(const floatx4 *)wp;
              w1 = *(const floatx4 *)(wp + 16);
            } else {
              // last chunk: staged columns 16 (KCH - 1) .. + 3 only (lane
              // group 0); the other groups read group 0's address
              const floatx4 v = *(const floatx4 *)(wp - 4 * g);
              w0 = g == 0 ? v : z;
              w1 = z;
            }
            w[nt] = to_bf16x8(w0, w1);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma_bf16x2(w[nt], xc[mt][p], acc[mt][nt]);
        }
        epi.template apply<MT, NT>(acc, row0, cb * NT, ntt, lane, M, cs + cb * NT * 16);
      }
      if (next) to_pairs();
    }
    return;
  }
  floatx4 xr[MT][KCH], xn[MT][KCH];
  if (row0 < M) load_x_tile<MT, KCH, 0, 1>(a, row0, M, r, g, xr);
  for (; row0 < M; row0 += stride) {
    if (row0 + stride < M) load_x_tile<MT, KCH, 0, 1>(a, row0 + stride, M, r, g, xn);
#pragma unroll 1
    for (int cb = 0; cb < CB; ++cb) {
      floatx4 acc[MT][NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
      const float *wb = wsm + (cb * NT * 16 + r) * LDW;
#pragma unroll
      for (int c = 0; c < KCH; ++c) {
        if (c == KCH - 1) {
          // one step: depth 16 c + g on both operands
          const float *wt = wb + 16 * c + g;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const float wv = wt[nt * 16 * LDW];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(wv, xr[mt][c][0], acc[mt][nt]);
          }
          continue;
        }
        floatx4 w[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) w[nt] = *(const floatx4 *)(wb + nt * 16 * LDW + 16 * c + 4 * g);
        __builtin_amdgcn_sched_barrier(0);  // one chunk of weights live at a time
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4(w[nt][t], xr[mt][c][t], acc[mt][nt]);
      }
      epi.template apply<MT, NT>(acc, row0, cb * NT, ntt, lane, M, cs + cb * NT * 16);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int c = 0; c < KCH; ++c) xr[mt][c] = xn[mt][c];
  }
}

// ------------------------------------------------------------------ epilogues
//
// Every epilogue issues all the global loads of a 16-row tile (clamped to
// valid rows and columns) before it uses any of them, and masks with selects:
// a load inside a branch, or a value used right after its load, makes the
// wavefront wait for that load alone, and a few dozen such waits cost more
// than the MFMAs of the tile.  Per-column vectors (bias, gamma, ...) are
// staged in LDS once per block: Epi::kCols of them over the block's NT*16
// columns, a null pointer staging zeros.  Optional row operands that a mode
// does not use read the zero table instead of branching around the load.

constexpr int kMaxCols = 3;
constexpr int kZeros = 4096;
__device__ float g_zeros[kZeros];  // zero-initialised, never written

struct EpiLinear {
  static constexpr int kLds = 1;  // LDS-weight kernel, next tile prefetched before the MFMAs
  static constexpr int kCols = 1;
  const float *bias;
  float *y;
  int ldy;
  int Nreal;
  int ybf16;  // 1: y is stored in BF16 (rounded to nearest even)
  __device__ __forceinline__ const float *col(int) const { return bias; }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *cs) const {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      if (row >= M) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (nt0 + nt >= ntt) continue;
        const floatx4 b = *(const floatx4 *)(cs + nt * 16 + 4 * g);
        const int n0 = (nt0 + nt) * 16 + 4 * g;
        floatx4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = n0 + v < Nreal ? acc[mt][nt][v] + b[v] : 0.f;
        if (ybf16)
          *(bf16x4 *)((__bf16 *)y + (size_t)row * ldy + n0) = to_bf16(o);
        else
          *(floatx4 *)(y + (size_t)row * ldy + n0) = o;
      }
    }
  }
};

// Split k: the raw partial sums of slice blockIdx.z, y + z * slice.
struct EpiPartial {
  static constexpr int kLds = 0;
  static constexpr int kCols = 1;
  float *y;
  int ldy;
  size_t slice;
  __device__ __forceinline__ const float *col(int) const { return nullptr; }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *) const {
    const int r = lane & 15, g = lane >> 4;
    float *yz = y + blockIdx.z * slice;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      if (row >= M) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (nt0 + nt >= ntt) continue;
        *(floatx4 *)(yz + (size_t)row * ldy + (nt0 + nt) * 16 + 4 * g) = acc[mt][nt];
      }
    }
  }
};

// y = tanh(acc + b) + res ; the bias is per column, or per row type when
// row_type is set (bias [ntypes][bias_ld], read from global memory).
struct EpiTanhRes {
  static constexpr int kLds = 0;  // streaming kernel only
  static constexpr int kCols = 1;
  const float *bias;
  const int32_t *row_type;
  int bias_ld;
  const float *res;
  int ldr;
  int res_mode;
  int res_fin;
  float *y;
  int ldy;
  float *tout;
  int ldt;
  int Nreal;
  __device__ __forceinline__ const float *col(int) const { return row_type ? nullptr : bias; }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *cs) const {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      const bool ok = row < M;
      const size_t rr = (size_t)(ok ? row : 0);
      floatx4 bl[NT], rv[NT];
      if (row_type) {
        const float *bp = bias + (size_t)row_type[rr] * bias_ld;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int tile = nt0 + nt < ntt ? nt0 + nt : 0;
          bl[nt] = *(const floatx4 *)(bp + tile * 16 + 4 * g);
        }
      } else {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bl[nt] = *(const floatx4 *)(cs + nt * 16 + 4 * g);
      }
      // residual: 16-byte loads for the identity rule, scalar ones for the
      // doubling rule (uniform branch; every load is issued before any use)
      if (res_mode == RES_IDENT) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int tile = nt0 + nt < ntt ? nt0 + nt : 0;
          rv[nt] = *(const floatx4 *)(res + rr * ldr + tile * 16 + 4 * g);
        }
      } else if (res_mode == RES_DOUBLE) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // doubling: Nreal = 2 res_fin, so n mod res_fin is one subtraction
            const int n = (nt0 + nt) * 16 + 4 * g + v;
            const int nn = n < Nreal ? n : 0;
            rv[nt][v] = res[rr * ldr + (nn >= res_fin ? nn - res_fin : nn)];
          }
      } else {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) rv[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
      if (!ok) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (nt0 + nt >= ntt) continue;
        const int n0 = (nt0 + nt) * 16 + 4 * g;
        floatx4 o, tv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool in = n0 + v < Nreal;
          const float t = tanh_fast(acc[mt][nt][v] + bl[nt][v]);
          o[v] = in ? t + rv[nt][v] : 0.f;
          tv[v] = in ? t : 0.f;
        }
        *(floatx4 *)(y + rr * ldy + n0) = o;
        if (tout) *(floatx4 *)(tout + rr * ldt + n0) = tv;
      }
    }
  }
};

// Output projection + layer norm + residual (all output columns in one wave).
struct EpiLNRes {
  static constexpr int kLds = 2;  // LDS-weight kernel, next tile prefetched after the MFMAs
  static constexpr int kCols = 3;
  const float *bias, *gamma, *beta;
  float eps;
  const float *gin;
  int ld;  // row stride of gin, gout, xhat (= Npad)
  float *gout, *xhat, *rstd;
  int Nreal;
  __device__ __forceinline__ const float *col(int k) const {
    return k == 0 ? bias : (k == 1 ? gamma : beta);
  }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *cs) const {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      const bool ok = row < M;
      const size_t rb = (size_t)(ok ? row : 0) * ld;
      floatx4 gi[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int tile = nt < ntt ? nt : 0;
        gi[nt] = *(const floatx4 *)(gin + rb + tile * 16 + 4 * g);
      }
      lnres::apply_tile<NT>(acc[mt], gi, g, ntt, Nreal, eps, cs, NT * 16, ok, row, rb, gout,
                            xhat, rstd);
    }
  }
};

// d = acc + residual gradient ; a = d * (1 - t^2).  The residual is a row
// operand (RES_IDENT, RES_FOLD) or a column vector (RES_BCAST).
struct EpiBwdTanh {
  static constexpr int kLds = 0;  // streaming kernel only
  static constexpr int kCols = 1;
  const float *res;
  int ldr;
  int res_mode;
  int res_fin;
  const float *t;
  int ldt;
  float *d;
  int ldd;
  float *aout;
  int lda;
  int Nreal;
  __device__ __forceinline__ const float *col(int) const {
    return res_mode == RES_BCAST ? res : nullptr;
  }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *cs) const {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      const bool ok = row < M;
      const size_t rr = (size_t)(ok ? row : 0);
      floatx4 tt[NT], rv[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int tile = nt0 + nt < ntt ? nt0 + nt : 0;
        tt[nt] = *(const floatx4 *)(t + rr * ldt + tile * 16 + 4 * g);
      }
      // row residual gradient: 16-byte loads for the identity rule, scalar
      // pairs for the folded doubling rule (uniform branch)
      if (res_mode == RES_IDENT) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int tile = nt0 + nt < ntt ? nt0 + nt : 0;
          rv[nt] = *(const floatx4 *)(res + rr * ldr + tile * 16 + 4 * g);
        }
      } else if (res_mode == RES_FOLD) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = (nt0 + nt) * 16 + 4 * g + v;
            const int nn = n < Nreal ? n : 0;
            rv[nt][v] = res[rr * ldr + nn] + res[rr * ldr + nn + res_fin];
          }
      } else {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) rv[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
      if (!ok) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (nt0 + nt >= ntt) continue;
        const int n0 = (nt0 + nt) * 16 + 4 * g;
        const floatx4 bc = *(const floatx4 *)(cs + nt * 16 + 4 * g);
        floatx4 dv, av;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool in = n0 + v < Nreal;
          const float x = acc[mt][nt][v] + rv[nt][v] + bc[v];
          dv[v] = in ? x : 0.f;
          av[v] = in ? x * (1.0f - tt[nt][v] * tt[nt][v]) : 0.f;
        }
        if (d) *(floatx4 *)(d + rr * ldd + n0) = dv;
        *(floatx4 *)(aout + rr * lda + n0) = av;
      }
    }
  }
};

// dgin = acc + dgout ; then layer-norm backward (mode 0), tanh backward
// (mode 1) or nothing (mode 2).
struct EpiQKVBwd {
  static constexpr int kLds = 0;  // streaming kernel only
  static constexpr int kCols = 1;
  const float *dgout;
  int mode;
  const float *gamma, *xhat, *rstd, *t;
  int ld;
  float *dgin, *dnext;
  int Nreal;
  __device__ __forceinline__ const float *col(int) const { return mode == 0 ? gamma : nullptr; }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *cs) const {
    const int r = lane & 15, g = lane >> 4;
    const float invn = 1.0f / (float)Nreal;
    // second row operand: xhat (mode 0) or t (mode 1); mode 2 rereads dgout
    const float *aux = mode == 0 ? xhat : (mode == 1 ? t : dgout);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      const bool ok = row < M;
      const size_t rb = (size_t)(ok ? row : 0) * ld;
      floatx4 go[NT], ax[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int tile = nt < ntt ? nt : 0;
        go[nt] = *(const floatx4 *)(dgout + rb + tile * 16 + 4 * g);
        ax[nt] = *(const floatx4 *)(aux + rb + tile * 16 + 4 * g);
      }
      const float rs = *(mode == 0 ? rstd + (ok ? row : 0) : g_zeros);
      float s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const floatx4 gm = *(const floatx4 *)(cs + nt * 16 + 4 * g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const bool in = nt < ntt && n < Nreal;
          acc[mt][nt][v] = in ? acc[mt][nt][v] + go[nt][v] : 0.f;
          const float dx = gm[v] * acc[mt][nt][v];
          s1 += dx;
          s2 += dx * ax[nt][v];
        }
      }
      const float m1 = row_sum16(s1) * invn;
      const float m2 = row_sum16(s2) * invn;
      if (!ok) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (nt >= ntt) continue;
        const int n0 = nt * 16 + 4 * g;
        *(floatx4 *)(dgin + rb + n0) = acc[mt][nt];
        if (mode == 2) continue;
        const floatx4 gm = *(const floatx4 *)(cs + n0);
        floatx4 dn;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool in = n0 + v < Nreal;
          const float ln = rs * (gm[v] * acc[mt][nt][v] - m1 - ax[nt][v] * m2);
          const float th = acc[mt][nt][v] * (1.0f - ax[nt][v] * ax[nt][v]);
          dn[v] = in ? (mode == 0 ? ln : th) : 0.f;
        }
        *(floatx4 *)(dnext + rb + n0) = dn;
      }
    }
  }
};

// dh1 = acc + residual(dh2); du1 = dh1 * (1 - h1^2); gs = sum_o du1[o] * ws[o]
struct EpiEmb1Bwd {
  static constexpr int kLds = 0;  // streaming kernel only
  static constexpr int kCols = 1;
  const float *dh2;
  int ldd2, res_mode, fin;
  const float *h1;
  int ldh1;
  const float *ws;
  float *gs;
  int Nreal;
  __device__ __forceinline__ const float *col(int) const { return ws; }
  template <int MT, int NT>
  __device__ __forceinline__ void apply(floatx4 (&acc)[MT][NT], int row0, int nt0, int ntt,
                                        int lane, int M, const float *cs) const {
    const int r = lane & 15, g = lane >> 4;
    const bool rowres = res_mode == RES_IDENT || res_mode == RES_FOLD;
    const float *rp = rowres ? dh2 : g_zeros;
    const int rld = rowres ? ldd2 : 0;
    const int fold = res_mode == RES_FOLD ? fin : 0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = row0 + mt * 16 + r;
      const bool ok = row < M;
      const size_t rr = (size_t)(ok ? row : 0);
      float hv[NT][4], r1[NT][4], r2[NT][4];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const int nn = (nt < ntt && n < Nreal) ? n : 0;
          hv[nt][v] = h1[rr * ldh1 + nn];
          r1[nt][v] = rp[rr * rld + nn];
          r2[nt][v] = rp[rr * rld + nn + fold];  // = r1 unless folding; masked at use
        }
      float s = 0.f;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const floatx4 wv = *(const floatx4 *)(cs + nt * 16 + 4 * g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + 4 * g + v;
          const float dd = acc[mt][nt][v] + r1[nt][v] + (fold ? r2[nt][v] : 0.f);
          const float term = dd * (1.0f - hv[nt][v] * hv[nt][v]) * wv[v];
          s += (nt < ntt && n < Nreal) ? term : 0.f;
        }
      }
      s = row_sum16(s);
      if (ok && g == 0) gs[row] = s;
    }
  }
};

// Stage the epilogue's column vectors for the block's column tiles into LDS:
// cs[k][j] = col(k)[nt0 * 16 + j] for j < NT * 16 (zero past Npad or for a
// null vector).  Called by every thread of the block, followed by a barrier.
template <class Epi, int NT>
__device__ void stage_cols(const Epi &e, int nt0, int npad, float *cs) {
  for (int idx = threadIdx.x; idx < Epi::kCols * NT * 16; idx += blockDim.x) {
    const int k = idx / (NT * 16), j = idx % (NT * 16);
    const int n = nt0 * 16 + j;
    const float *p = e.col(k);
    cs[idx] = (p != nullptr && n < npad) ? p[n] : 0.f;
  }
}

int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

// Grid of the streaming kernel: one block per 4*16*MT rows, capped at the
// number of blocks the device holds at once (the kernel loops over tiles).
template <int MT, int NT, class Epi, int BF>
void launch_stream_p(const GemmArgs &a, const Epi &e, unsigned gy, hipStream_t s) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_gemm<MT, NT, Epi, BF>, 256, 0) !=
            hipSuccess ||
        nb <= 0)
      nb = 2;
    per_cu = nb;
  }
  const long tiles = (a.Mmax + 64 * MT - 1) / (64 * MT);
  long cap = (long)per_cu * cu_count() / (long)gy;
  if (cap < 1) cap = 1;
  const unsigned gx = (unsigned)(tiles < cap ? tiles : cap);
  if (gx == 0) return;
  hipLaunchKernelGGL((k_gemm<MT, NT, Epi, BF>), dim3(gx, gy), dim3(256), 0, s, a, e);
}
template <int MT, int NT, class Epi>
void launch_stream(const GemmArgs &a, const Epi &e, unsigned gy, hipStream_t s) {
  if (a.bf16 && a.xbf16) launch_stream_p<MT, NT, Epi, 2>(a, e, gy, s);
  else if (a.bf16) launch_stream_p<MT, NT, Epi, 1>(a, e, gy, s);
  else launch_stream_p<MT, NT, Epi, 0>(a, e, gy, s);
}

template <class Epi, int MT>
void dispatch_nt(const GemmArgs &a, const Epi &e, int nt, hipStream_t s) {
  const int ntt = a.Npad / 16;
  const unsigned gy = (unsigned)((ntt + nt - 1) / nt);
  switch (nt) {
    case 1: launch_stream<MT, 1>(a, e, gy, s); break;
    case 2: launch_stream<MT, 2>(a, e, gy, s); break;
    case 3: launch_stream<MT, 3>(a, e, gy, s); break;
    case 4: launch_stream<MT, 4>(a, e, gy, s); break;
    case 5: launch_stream<MT, 5>(a, e, gy, s); break;
    case 6: launch_stream<MT, 6>(a, e, gy, s); break;
    case 7: launch_stream<MT, 7>(a, e, gy, s); break;
    default: launch_stream<MT, 8>(a, e, gy, s); break;
  }
}

// LDS bytes of the resident-weight kernel: W^T[Nreal][K + 4] and the staged
// column vectors.
template <class Epi, int NT, int KCH>
size_t wres_lds(int nreal) {
  return sizeof(float) * ((size_t)nreal * (KCH * 16 + 4) + Epi::kCols * NT * 16);
}

// One workgroup of eight wavefronts per CU; the grid never exceeds the CU
// count (a second wave of workgroups would start only after the first).
template <class Epi, int NT, int KCH>
bool launch_wres(const GemmArgs &a, const Epi &e, hipStream_t s) {
  constexpr int MT = 4;
  static int ready[64];  // 1: dynamic LDS limit raised on that device, -1: refused
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  const size_t lds = wres_lds<Epi, NT, KCH>(a.Nreal);
  if (ready[dev] == 0) {
    int maxl = 0;
    ready[dev] = hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                             hipSuccess &&
                         hipFuncSetAttribute((const void *)k_gemm_wres<MT, NT, KCH, Epi>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             maxl) == hipSuccess
                     ? maxl
                     : -1;
  }
  if (ready[dev] < 0 || lds > (size_t)ready[dev]) return false;
  const long tiles = (a.Mmax + 8L * 16 * MT - 1) / (8L * 16 * MT);
  const long gx = tiles < cu_count() ? tiles : cu_count();
  if (gx <= 0) return true;
  hipLaunchKernelGGL((k_gemm_wres<MT, NT, KCH, Epi>), dim3((unsigned)gx), dim3(512), lds, s, a, e);
  return true;
}

// One workgroup of eight wavefronts per CU (the grid never exceeds the CU
// count).  Returns false when the weight block does not fit the device's LDS.
template <class Epi, int NT, int CB, int KCH, int BF>
bool launch_cols(const GemmArgs &a, const Epi &e, hipStream_t s) {
  constexpr int KS = 16 * (KCH - 1) + 4, NC = CB * NT * 16;
  static int ready[64];  // dynamic LDS limit: 0 unknown, -1 refused, else bytes
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  const size_t lds = sizeof(float) * ((size_t)NC * (KS + 4) + NC);
  if (ready[dev] == 0) {
    int maxl = 0;
    ready[dev] = hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                             hipSuccess &&
                         hipFuncSetAttribute((const void *)k_gemm_cols<NT, CB, KCH, Epi, BF>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             maxl) == hipSuccess
                     ? maxl
                     : -1;
  }
  if (ready[dev] < 0 || lds > (size_t)ready[dev]) return false;
  const long tiles = (a.Mmax + 8L * 32 - 1) / (8L * 32);
  const long gx = tiles < cu_count() ? tiles : cu_count();
  if (gx <= 0) return true;
  hipLaunchKernelGGL((k_gemm_cols<NT, CB, KCH, Epi, BF>), dim3((unsigned)gx), dim3(512), lds, s,
                     a, e);
  return true;
}

template <class Epi, int NT, int KCH>
void launch_lds(const GemmArgs &a, const Epi &e, hipStream_t s) {
  constexpr int MT = 2;
  const int ntt = a.Npad / 16;
  const unsigned gy = (unsigned)((ntt + NT - 1) / NT);
  const int row_tiles = (a.Mmax + 64 * MT - 1) / (64 * MT);
  // two workgroups per CU are resident (LDS and registers); the grid must not
  // exceed that, or the blocks past it start only when others have finished
  // their whole share and the launch takes twice as long
  int gx = 2 * cu_count() / (int)gy / 8 * 8;
  if (gx < 8) gx = 8;
  if (gx > row_tiles) gx = (row_tiles + 7) / 8 * 8;
  if (gx <= 0) return;
  const size_t lds = sizeof(float) * NT * 16 * (KCH * 16 + 4 + Epi::kCols);
  // FP32 with data only in the first four columns of the last chunk
  const bool short_tail = a.kreal > 16 * (KCH - 1) && a.kreal <= 16 * (KCH - 1) + 4;
  if (a.bf16 && a.xbf16)
    hipLaunchKernelGGL((k_gemm_lds<MT, NT, KCH, Epi, 2, 4>), dim3(gx, gy), dim3(256), lds, s, a, e);
  else if (a.bf16)
    hipLaunchKernelGGL((k_gemm_lds<MT, NT, KCH, Epi, 1, 4>), dim3(gx, gy), dim3(256), lds, s, a, e);
  else if (short_tail)
    hipLaunchKernelGGL((k_gemm_lds<MT, NT, KCH, Epi, 0, 1>), dim3(gx, gy), dim3(256), lds, s, a, e);
  else
    hipLaunchKernelGGL((k_gemm_lds<MT, NT, KCH, Epi, 0, 4>), dim3(gx, gy), dim3(256), lds, s, a, e);
}

// Split k, second pass: each lane adds its tile values over the slices in
// slice order and applies the product's own epilogue to the sums.
template <int NT, class Epi>
__global__ __launch_bounds__(256) void k_splitk_finish(const float *__restrict__ part, int nslice,
                                                     size_t slice, int ldp, int M, int Npad,
                                                     Epi epi) {
  __shared__ float cs[Epi::kCols * NT * 16];
  const int nt0 = blockIdx.y * NT;
  stage_cols<Epi, NT>(epi, nt0, Npad, cs);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int row0 = (blockIdx.x * 4 + wave) * 16;
  if (row0 >= M) return;  // no barrier follows
  const int ntt = Npad / 16;
  const size_t rb = (size_t)(row0 + r < M ? row0 + r : 0) * ldp;
  floatx4 acc[1][NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int tile = nt0 + nt < ntt ? nt0 + nt : 0;
    acc[0][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int z = 0; z < nslice; ++z)
      acc[0][nt] += *(const floatx4 *)(part + z * slice + rb + tile * 16 + 4 * g);
  }
  epi.template apply<1, NT>(acc, row0, nt0, ntt, lane, M, cs);
}

// Rows per wave: two 16-row tiles for the large pair-batched products,
// one for the centre-batched fitting net (more blocks for fewer rows).
template <class Epi>
void run(const GemmArgs &a, const Epi &e, bool full_rows, hipStream_t s) {
  const int ntt = a.Npad / 16;
  int nt = ntt < 8 ? ntt : 8;
  if (full_rows && ntt > 8) nt = ntt;  // callers guarantee ntt <= 8 for row reductions
  // per-centre products (the fitting net: few rows, long k loops) run on
  // column blocks of at most four tiles: more wavefronts per SIMD to cover
  // the load latency of each k step (measured best against 1, 2 and 8)
  if (!full_rows && a.Mmax < 65536 && nt > 4) nt = 4;
  // the FP32 QKV projection (384 output columns over a 100-wide embedding):
  // the whole weight block resident, X read once
  if constexpr (Epi::kLds == 1 && Epi::kCols == 1) {
    if (a.Mmax >= 65536 && !(a.bf16 && a.xbf16) && a.K == 112 && ntt == 24 && a.kreal > 96 &&
        a.kreal <= 100 &&
        (a.bf16 ? launch_cols<Epi, 8, 3, 7, 1>(a, e, s) : launch_cols<Epi, 8, 3, 7, 0>(a, e, s)))
      return;
  }
  if constexpr (Epi::kLds != 0) {
    if (a.Mmax >= 65536 && (a.K == 112 || a.K == 128) && (nt == 7 || nt == 8)) {
      if (nt == 7 && a.K == 112) return launch_lds<Epi, 7, 7>(a, e, s);
      if (nt == 7 && a.K == 128) return launch_lds<Epi, 7, 8>(a, e, s);
      if (nt == 8 && a.K == 112) return launch_lds<Epi, 8, 7>(a, e, s);
      return launch_lds<Epi, 8, 8>(a, e, s);
    }
  }
  // the FP32 adjoint of the QKV projection (K = 384, seven column tiles):
  // the whole weight block resident in LDS when it fits
  if constexpr (Epi::kLds == 0) {
    if (a.Mmax >= 65536 && full_rows && !a.bf16 && a.K == 384 && nt == 7 && ntt == 7 &&
        launch_wres<Epi, 7, 24>(a, e, s))
      return;
  }
  // the long-K adjoint of the QKV projection otherwise: 64-row tiles halve
  // the weight reads per row (two waves per SIMD, 238 registers, no spills)
  if (a.Mmax >= 65536 && full_rows && Epi::kLds == 0 && a.K >= 256) dispatch_nt<Epi, 4>(a, e, nt, s);
  else if (a.Mmax >= 65536) dispatch_nt<Epi, 2>(a, e, nt, s);
  else dispatch_nt<Epi, 1>(a, e, nt, s);
}

}  // namespace

void gemm_linear(const GemmArgs &a, const float *bias, float *y, int ldy, hipStream_t s,
                 int ybf16) {
  EpiLinear e{bias, y, ldy, a.Nreal, ybf16};
  run(a, e, false, s);
}

void gemm_tanh_res(const GemmArgs &a, const float *bias, const int32_t *row_type, int bias_ld,
                   const float *res, int ldr, int res_mode, int res_fin, float *y, int ldy,
                   float *tout, int ldt, hipStream_t s) {
  EpiTanhRes e{bias, row_type, bias_ld, res, ldr, res_mode, res_fin, y, ldy, tout, ldt, a.Nreal};
  run(a, e, false, s);
}

bool gemm_tanh_res_split(const GemmArgs &a, const float *bias, const int32_t *row_type,
                         int bias_ld, float *y, int ldy, float *tout, int ldt, float *scratch,
                         size_t scratch_floats, hipStream_t s) {
  // few rows: fewer than 64 row blocks of 64, so the unsplit product would
  // occupy a fraction of the CUs for the whole k loop
  constexpr int kMaxRows = 4096, kSlices = 8, NT = 4;
  const int M = a.Mmax;
  if (a.Mptr || M <= 0 || M >= kMaxRows || a.K < 512 || (a.bf16 && a.xbf16) || !scratch)
    return false;
  const int kslice = ((a.K + kSlices - 1) / kSlices + 31) / 32 * 32;  // whole 32-deep chunks
  const int nslice = (a.K + kslice - 1) / kslice;
  const size_t slice = (size_t)M * a.Npad;
  if ((size_t)nslice * slice > scratch_floats) return false;
  GemmArgs as = a;
  as.kslice = kslice;
  as.kreal = 0;
  const EpiPartial ep{scratch, a.Npad, slice};
  const int ntt = a.Npad / 16;
  const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((ntt + NT - 1) / NT), (unsigned)nslice);
  if (a.bf16)
    hipLaunchKernelGGL((k_gemm<1, NT, EpiPartial, 1>), grid, dim3(256), 0, s, as, ep);
  else
    hipLaunchKernelGGL((k_gemm<1, NT, EpiPartial, 0>), grid, dim3(256), 0, s, as, ep);
  const EpiTanhRes e{bias, row_type, bias_ld, nullptr, 0, RES_NONE, 0, y, ldy, tout, ldt, a.Nreal};
  hipLaunchKernelGGL((k_splitk_finish<NT, EpiTanhRes>), dim3(grid.x, grid.y), dim3(256), 0, s,
                     scratch, nslice, slice, a.Npad, M, a.Npad, e);
  return true;
}

void gemm_ln_res(const GemmArgs &a, const float *bias, const float *gamma, const float *beta,
                 float eps, const float *gin, int ldg, float *gout, float *xhat, float *rstd,
                 hipStream_t s) {
  EpiLNRes e{bias, gamma, beta, eps, gin, ldg, gout, xhat, rstd, a.Nreal};
  run(a, e, true, s);
}

void gemm_bwd_tanh(const GemmArgs &a, const float *res, int ldr, int res_mode, int res_fin,
                   const float *t, int ldt, float *d, int ldd, float *aout, int lda,
                   hipStream_t s) {
  EpiBwdTanh e{res, ldr, res_mode, res_fin, t, ldt, d, ldd, aout, lda, a.Nreal};
  run(a, e, false, s);
}

void gemm_qkv_bwd(const GemmArgs &a, const float *dgout, int mode, const float *gamma,
                  const float *xhat, const float *rstd, const float *t, float *dgin,
                  float *dnext, hipStream_t s) {
  EpiQKVBwd e{dgout, mode, gamma, xhat, rstd, t, a.Npad, dgin, dnext, a.Nreal};
  run(a, e, true, s);
}

void gemm_emb1_bwd(const GemmArgs &a, const float *dh2, int ldd2, int res_mode, int fin,
                   const float *h1, int ldh1, const float *ws, float *gs, hipStream_t s) {
  EpiEmb1Bwd e{dh2, ldd2, res_mode, fin, h1, ldh1, ws, gs, a.Nreal};
  run(a, e, true, s);
}

}  // namespace dpa1
