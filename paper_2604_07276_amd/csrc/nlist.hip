// Neighbour search and per-pair geometry for DPA-1 inference on gfx950.
//
// Full neighbour lists within the cutoff (Sec. II-A: cutoff lists make the
// cost O(N); Sec. II-C: a DP descriptor needs the full list of every centre).
// A cell grid with edge >= rcut bins the atoms; one workgroup per cell
// stages the candidates of the 27 surrounding cells in LDS, and one
// wavefront per centre tests them in FP64 and compacts hits with a ballot.  Lists are sorted by atom index so that every later stage
// sees a deterministic neighbour order.
//
// Pair vectors follow one fixed FP64 recipe, with contraction disabled so
// the result does not depend on FMA formation:
//   d = x_j - x_i;  with a box d -= L * rint(d / L);
//   r2 = (dx*dx + dy*dy) + dz*dz;  neighbour iff r2 < rcut*rcut.
#include <climits>

#include "dpa1_internal.h"

namespace dpa1 {

namespace {

constexpr int kWave = 64;
constexpr int kListCap = 128;      // == DP_MAX_SEL

__device__ __forceinline__ void pair_vec(const double *__restrict__ x, int i, int j,
                                         const CellGrid &g, double d[3]) {
#pragma clang fp contract(off)
  for (int c = 0; c < 3; ++c) {
    double v = x[3 * j + c] - x[3 * i + c];
    if (g.periodic) v = v - g.L[c] * rint(v / g.L[c]);
    d[c] = v;
  }
}

__device__ __forceinline__ double norm2(const double d[3]) {
#pragma clang fp contract(off)
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

__device__ __forceinline__ int cell_coord(double x, int c, const CellGrid &g) {
  double u;
  if (g.periodic) {
    double w = x - g.L[c] * floor(x / g.L[c]);
    u = w * g.inv_edge[c];
  } else {
    u = (x - g.lo[c]) * g.inv_edge[c];
  }
  int k = (int)floor(u);
  k = k < 0 ? 0 : k;
  k = k >= g.nc[c] ? g.nc[c] - 1 : k;
  return k;
}

// Flags out-of-range types and writes a clamped copy that every later kernel
// indexes tables with, so a bad input can never address outside them.
__global__ void k_check_types(const int32_t *__restrict__ types, int nall, int ntypes,
                              DevFlags *flags, int32_t *__restrict__ safe) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nall) return;
  int t = types[k];
  if (t < 0 || t >= ntypes) {
    atomicMin(&flags->bad_type_atom, k);
    t = t < 0 ? 0 : ntypes - 1;
  }
  safe[k] = t;
}

__global__ void k_cell_bin(const double *__restrict__ x, int nall, CellGrid g,
                           int *__restrict__ atom_cell, int *__restrict__ cell_count) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nall) return;
  int cx = cell_coord(x[3 * k + 0], 0, g);
  int cy = cell_coord(x[3 * k + 1], 1, g);
  int cz = cell_coord(x[3 * k + 2], 2, g);
  int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
  atom_cell[k] = c;
  atomicAdd(&cell_count[c], 1);
}

// Single-block exclusive scan: out[0..n) exclusive prefix sums, out[n] total.
// Thread t owns the contiguous chunk [t per, (t + 1) per); its loads are
// issued eight at a time, and the chunk totals are scanned within each
// wavefront with shuffles and across the sixteen wavefronts in LDS.
__global__ __launch_bounds__(1024) void k_scan(const int *__restrict__ in, int n,
                                               int *__restrict__ out) {
  __shared__ int wtot[16];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int per = (n + 1023) / 1024;
  const int b = t * per;
  const int e = min(b + per, n);
  int s = 0;
  for (int k0 = b; k0 < e; k0 += 8) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k0 + u < e ? in[k0 + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  // inclusive scan of the chunk totals within the wavefront
  int inc = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wtot[wave] = inc;
  __syncthreads();
  int before = 0;  // totals of the earlier wavefronts
  for (int w = 0; w < wave; ++w) before += wtot[w];
  int run = before + inc - s;  // exclusive prefix of this chunk
  for (int k0 = b; k0 < e; k0 += 8) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k0 + u < e ? in[k0 + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u < e) out[k0 + u] = run;
      run += v[u];
    }
  }
  if (t == 1023) out[n] = before + inc;
}

__global__ void k_cell_fill(const int *__restrict__ atom_cell, int nall,
                            const int *__restrict__ cell_start, int *__restrict__ cell_fill,
                            int *__restrict__ cell_atoms) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nall) return;
  int c = atom_cell[k];
  int pos = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + pos] = k;
}

// Distinct cell offsets along one dimension.
__device__ __forceinline__ int dim_offsets(const CellGrid &g, int dim, int c, int out[3]) {
  int n = 0;
  const int nc = g.nc[dim];
  if (g.periodic) {
    if (nc >= 3) {
      out[n++] = (c + nc - 1) % nc;
      out[n++] = c;
      out[n++] = (c + 1) % nc;
    } else if (nc == 2) {
      out[n++] = 0;
      out[n++] = 1;
    } else {
      out[n++] = 0;
    }
  } else {
    for (int o = -1; o <= 1; ++o) {
      int q = c + o;
      if (q >= 0 && q < nc) out[n++] = q;
    }
  }
  return n;
}

// One workgroup per cell.  Every atom of a cell has the same 27 neighbour
// cells, so the workgroup stages their candidates (atom index and FP64
// coordinates) in LDS once and each wavefront then tests its centres (one
// at a time) against the staged tile, 64 candidates per pass.  Local
// centres collect every atom within rcut; ghost centres collect local atoms
// only (they are needed by the force gather, never as energy centres).  A
// neighbourhood with more candidates than the tile holds is scanned from
// global memory instead (same ranges, same test).
constexpr int kCellWaves = 8;      // wavefronts per cell workgroup
constexpr int kTileCap = 1536;     // staged candidates (about 2.5x the protein density)
constexpr int kMaxRanges = 27;

// The pair test on FP64 coordinates: the recipe of pair_vec and norm2.
__device__ __forceinline__ bool within(double xi0, double xi1, double xi2, double xj0, double xj1,
                                       double xj2, const CellGrid &g, double rc2) {
#pragma clang fp contract(off)
  double d0 = xj0 - xi0, d1 = xj1 - xi1, d2 = xj2 - xi2;
  if (g.periodic) {
    d0 = d0 - g.L[0] * rint(d0 / g.L[0]);
    d1 = d1 - g.L[1] * rint(d1 / g.L[1]);
    d2 = d2 - g.L[2] * rint(d2 / g.L[2]);
  }
  return (d0 * d0 + d1 * d1) + d2 * d2 < rc2;
}

__global__ __launch_bounds__(kWave *kCellWaves) void k_nlist(
    const double *__restrict__ x, int nloc, CellGrid g, double rc2, int sel,
    const int *__restrict__ cell_start, const int *__restrict__ cell_atoms,
    int *__restrict__ nlist, int *__restrict__ nnei, DevFlags *flags) {
  __shared__ int tj[kTileCap];
  __shared__ double tx[kTileCap], ty[kTileCap], tz[kTileCap];
  __shared__ int list[kCellWaves][kListCap];
  __shared__ int rb[kMaxRanges], roff[kMaxRanges + 1];
  __shared__ int nr;
  const int cell = blockIdx.x;
  const int a0 = cell_start[cell], a1 = cell_start[cell + 1];
  if (a0 == a1) return;  // empty cell: the whole workgroup leaves
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (threadIdx.x == 0) {
    // The cells of one (y, z) row are consecutive in the cell order, so their
    // atoms are one contiguous range of cell_atoms unless the row wraps: the
    // row's cells are visited in ascending index and merged while their
    // atom ranges touch.
    const int cx = cell % g.nc[0];
    const int cy = (cell / g.nc[0]) % g.nc[1];
    const int cz = cell / (g.nc[0] * g.nc[1]);
    int ox[3], oy[3], oz[3];
    const int nx = dim_offsets(g, 0, cx, ox);
    const int ny = dim_offsets(g, 1, cy, oy);
    const int nz = dim_offsets(g, 2, cz, oz);
    int q = 0, tot = 0;
    auto add = [&](int beg, int end) {
      rb[q] = beg;
      roff[q] = tot;
      tot += end - beg;
      ++q;
    };
    for (int a = 0; a < nz; ++a)
      for (int b = 0; b < ny; ++b) {
        const int row = (oz[a] * g.nc[1] + oy[b]) * g.nc[0];
        int cs[3];
        for (int c = 0; c < nx; ++c) cs[c] = row + ox[c];
        if (nx > 1 && cs[0] > cs[1]) { const int t = cs[0]; cs[0] = cs[1]; cs[1] = t; }
        if (nx > 2 && cs[1] > cs[2]) { const int t = cs[1]; cs[1] = cs[2]; cs[2] = t; }
        if (nx > 1 && cs[0] > cs[1]) { const int t = cs[0]; cs[0] = cs[1]; cs[1] = t; }
        int beg = cell_start[cs[0]], end = cell_start[cs[0] + 1];
        for (int c = 1; c < nx; ++c) {
          const int cb = cell_start[cs[c]], ce = cell_start[cs[c] + 1];
          if (cb == end) {
            end = ce;
          } else {
            add(beg, end);
            beg = cb;
            end = ce;
          }
        }
        add(beg, end);
      }
    roff[q] = tot;
    nr = q;
  }
  __syncthreads();
  const int R = nr;
  const int T = roff[R];
  const bool staged = T <= kTileCap;
  if (staged) {
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
      int q = 0;
      while (t >= roff[q + 1]) ++q;  // ranges are few (at most 27)
      const int j = cell_atoms[rb[q] + (t - roff[q])];
      tj[t] = j;
      tx[t] = x[3 * j + 0];
      ty[t] = x[3 * j + 1];
      tz[t] = x[3 * j + 2];
    }
  }
  __syncthreads();
  for (int ai = a0 + wave; ai < a1; ai += kCellWaves) {
    const int k = cell_atoms[ai];
    const bool ghost = k >= nloc;
    const double xk0 = x[3 * k + 0], xk1 = x[3 * k + 1], xk2 = x[3 * k + 2];
    int count = 0;
    auto keep = [&](bool hit, int j) {
      const unsigned long long m = __ballot(hit);
      const int pos = count + __popcll(m & ((1ull << lane) - 1ull));
      if (hit && pos < kListCap) list[wave][pos] = j;
      count += __popcll(m);
    };
    if (staged) {
      for (int base = 0; base < T; base += kWave) {
        const int t = base + lane;
        bool hit = false;
        int j = -1;
        if (t < T) {
          j = tj[t];
          if (j != k && (!ghost || j < nloc))
            hit = within(xk0, xk1, xk2, tx[t], ty[t], tz[t], g, rc2);
        }
        keep(hit, j);
      }
    } else {
      for (int q = 0; q < R; ++q) {
        const int beg = rb[q], end = rb[q] + (roff[q + 1] - roff[q]);
        for (int base = beg; base < end; base += kWave) {
          const int idx = base + lane;
          bool hit = false;
          int j = -1;
          if (idx < end) {
            j = cell_atoms[idx];
            if (j != k && (!ghost || j < nloc))
              hit = within(xk0, xk1, xk2, x[3 * j + 0], x[3 * j + 1], x[3 * j + 2], g, rc2);
          }
          keep(hit, j);
        }
      }
    }
    const int n = count < sel ? count : sel;
    if (count > sel) {
      if (lane == 0) {
        int old = atomicMin(&flags->overflow_atom, k);
        if (old > k) atomicExch(&flags->overflow_count, count);
      }
    }
    // rank sort of the (distinct) indices
    int vals[2], ranks[2];
    for (int h = 0; h < 2; ++h) {
      const int p = lane + h * kWave;
      vals[h] = p < n ? list[wave][p] : INT_MAX;
      ranks[h] = 0;
    }
    for (int q = 0; q < n; ++q) {
      const int v = list[wave][q];
      ranks[0] += v < vals[0];
      ranks[1] += v < vals[1];
    }
    int *row = nlist + (size_t)k * sel;
    for (int h = 0; h < 2; ++h) {
      const int p = lane + h * kWave;
      if (p < n) row[ranks[h]] = vals[h];
      else if (p < sel) row[p] = -1;
    }
    if (lane == 0) nnei[k] = n;
    __builtin_amdgcn_wave_barrier();  // the wave's list is rewritten by its next centre
  }
}

// One thread per (centre, slot).  Geometry in FP64, stored as FP32.
// One wavefront per centre: lane l handles slots l, l + 64 of the centre's
// list, so the pair records (contiguous per centre) are written by
// consecutive lanes, and each lane writes its h1 row with 16-byte stores.
// The type-pair table and ws are staged in LDS once per block (when they
// fit), so no global load sits inside the per-element loop.
constexpr int kEnvWaves = 4;
constexpr int kEnvTable = 8192;  // floats of type table staged in LDS

__global__ __launch_bounds__(kEnvWaves * 64) void k_env_embed1(
    const double *__restrict__ x, const int32_t *__restrict__ types, CellGrid g, int nloc,
    int sel, double rcut, double rs, const int *__restrict__ nlist, const int *__restrict__ nnei,
    const int *__restrict__ pair_off, const float *__restrict__ type_table,
    const float *__restrict__ ws, int ntypes, int n1, int ld1, float *__restrict__ geom,
    float *__restrict__ h1) {
  __shared__ float tab_s[kEnvTable];
  __shared__ float ws_s[128];
  const int tsize = ntypes * ntypes * ld1;
  const bool staged = tsize <= kEnvTable && ld1 <= 128;
  if (staged) {
    for (int k = threadIdx.x; k < tsize; k += blockDim.x) tab_s[k] = type_table[k];
    for (int k = threadIdx.x; k < ld1; k += blockDim.x) ws_s[k] = ws[k];
  }
  __syncthreads();
  const float *tab = staged ? tab_s : type_table;
  const float *wsv = staged ? ws_s : ws;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kEnvWaves + wave;
  if (i >= nloc) return;
  const int n = nnei[i];
  const int base = pair_off[i];
  const int ti = types[i];
  const double inv = 1.0 / (rcut - rs);
  for (int sl = lane; sl < n; sl += 64) {
    const int j = nlist[(size_t)i * sel + sl];
    const int tj = types[j];
    const int p = base + sl;
    double d[3];
    pair_vec(x, i, j, g, d);
    const double r = sqrt(norm2(d));
    // sw = u^3 (-6u^2 + 15u - 10) + 1 on [rs, rcut); dsw/dr = -30 u^2 (u - 1)^2 / (rcut - rs)
    const double u = (r - rs) * inv;
    const double swm = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0;
    const double dswm = -30.0 * u * u * (u - 1.0) * (u - 1.0) * inv;
    const double sw = r < rs ? 1.0 : (r < rcut ? swm : 0.0);
    const double dsw = (r < rs || r >= rcut) ? 0.0 : dswm;
    const double sv = sw / r;
    float4 *gp = (float4 *)(geom + (size_t)p * kGeom);
    gp[0] = make_float4((float)sv, (float)(d[0] / r), (float)(d[1] / r), (float)(d[2] / r));
    // slot 7: FP32 remainder of sw (the FP32 attention logits take hi + lo in FP64)
    gp[1] = make_float4((float)sw, (float)r, (float)dsw, (float)(sw - (double)(float)sw));
    const float s32 = (float)sv;
    const float *tt = tab + ((size_t)tj * ntypes + ti) * ld1;
    float4 *hp = (float4 *)(h1 + (size_t)p * ld1);
    for (int o = 0; o < ld1; o += 4) {
      float4 v;
      v.x = o + 0 < n1 ? tanh_fast(tt[o + 0] + wsv[o + 0] * s32) : 0.0f;
      v.y = o + 1 < n1 ? tanh_fast(tt[o + 1] + wsv[o + 1] * s32) : 0.0f;
      v.z = o + 2 < n1 ? tanh_fast(tt[o + 2] + wsv[o + 2] * s32) : 0.0f;
      v.w = o + 3 < n1 ? tanh_fast(tt[o + 3] + wsv[o + 3] * s32) : 0.0f;
      hp[o >> 2] = v;
    }
  }
}

}  // namespace

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_check_types(const int32_t *types, int nall, int ntypes, DevFlags *flags,
                        int32_t *safe, hipStream_t s) {
  if (nall <= 0) return;
  hipLaunchKernelGGL(k_check_types, dim3(nblk(nall, 256)), dim3(256), 0, s, types, nall, ntypes,
                     flags, safe);
}

void launch_cell_bin(const double *coords, int nall, CellGrid grid, int *atom_cell,
                     int *cell_count, hipStream_t s) {
  if (nall <= 0) return;
  hipLaunchKernelGGL(k_cell_bin, dim3(nblk(nall, 256)), dim3(256), 0, s, coords, nall, grid,
                     atom_cell, cell_count);
}

void launch_scan(const int *in, int n, int *out_excl, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, in, n, out_excl);
}

void launch_cell_fill(const int *atom_cell, int nall, const int *cell_start, int *cell_fill,
                      int *cell_atoms, hipStream_t s) {
  if (nall <= 0) return;
  hipLaunchKernelGGL(k_cell_fill, dim3(nblk(nall, 256)), dim3(256), 0, s, atom_cell, nall,
                     cell_start, cell_fill, cell_atoms);
}

void launch_nlist(const double *coords, int nloc, int nall, CellGrid grid, double rcut, int sel,
                  const int *cell_start, const int *cell_atoms, int *nlist, int *nnei,
                  DevFlags *flags, hipStream_t s) {
  if (nall <= 0) return;
  const int ncell = grid.nc[0] * grid.nc[1] * grid.nc[2];
  hipLaunchKernelGGL(k_nlist, dim3(ncell), dim3(kWave * kCellWaves), 0, s, coords, nloc, grid,
                     rcut * rcut, sel, cell_start, cell_atoms, nlist, nnei, flags);
}

void launch_env_embed1(const double *coords, const int32_t *types, CellGrid grid, int nloc,
                       int sel, double rcut, double rcut_smth, const int *nlist, const int *nnei,
                       const int *pair_off, const float *type_table, const float *ws, int ntypes,
                       int n1, int ld1, float *geom, float *h1, hipStream_t s) {
  if (nloc <= 0) return;
  hipLaunchKernelGGL(k_env_embed1, dim3(nblk(nloc, kEnvWaves)), dim3(kEnvWaves * 64), 0, s, coords,
                     types, grid, nloc, sel, rcut, rcut_smth, nlist, nnei, pair_off, type_table,
                     ws, ntypes, n1, ld1, geom, h1);
}

}  // namespace dpa1
