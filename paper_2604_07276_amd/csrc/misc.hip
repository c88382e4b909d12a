// Atomic energies, per-pair position gradients, forces and virial.
//
// E = sum over local centres of e_i (Eq. (5)); F = -dE/dx (Eq. (2)).  With
// g_ij = de_i/dd_ij and d_ij = x_j - x_i the force on atom k is
//   F_k = [k local] sum_j g_kj - sum_{i local, k in N(i)} g_ik,
// which gives ghost atoms the force -sum_i de_i/dx_ghost that the caller
// reduces onto the owning domain (Sec. II-C, Eq. (7)).  The second sum is a
// gather over k's own full list: neighbour relations are symmetric (the
// pair distance is computed identically both ways), and k's slot in the
// sorted list of i is found by binary search, so no atomics are needed and
// the result is bit-reproducible.
#include "dpa1_internal.h"

namespace dpa1 {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ void pair_vec(const double *__restrict__ x, int i, int j,
                                         const CellGrid &g, double d[3]) {
#pragma clang fp contract(off)
  for (int c = 0; c < 3; ++c) {
    double v = x[3 * j + c] - x[3 * i + c];
    if (g.periodic) v = v - g.L[c] * rint(v / g.L[c]);
    d[c] = v;
  }
}

// one wavefront per centre row: e_i and the fitting-net adjoint seed
__global__ __launch_bounds__(256) void k_energy(const float *__restrict__ z3,
                                                const float *__restrict__ t3, int ld, int nfit,
                                                const float *__restrict__ w_out, float b_out,
                                                const float *__restrict__ ebias,
                                                const int32_t *__restrict__ types, int nloc,
                                                float *__restrict__ e, float *__restrict__ a3) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  if (i >= nloc) return;
  float s = 0.f;
  for (int c = lane; c < ld; c += kWave) {
    float a = 0.f;
    if (c < nfit) {
      const float w = w_out[c];
      s += z3[(size_t)i * ld + c] * w;
      const float t = t3[(size_t)i * ld + c];
      a = w * (1.0f - t * t);
    }
    a3[(size_t)i * ld + c] = a;
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) e[i] = s + b_out + ebias[types[i]];
}

// g_ij from the upstream gradients of one pair:
//   gs  dE/ds through the embedding input, dRt dE/dR~, gw dE/dsw (attention),
//   gr  dE/drhat (attention gate).
__global__ void k_env_bwd(const float *__restrict__ geom, const float *__restrict__ gs,
                          const float *__restrict__ dRt, const float *__restrict__ gw,
                          const float *__restrict__ gr, const int *__restrict__ Mptr,
                          float *__restrict__ gout) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *Mptr) return;
  const float *gp = geom + (size_t)p * kGeom;
  const float s = gp[G_S], rx = gp[G_RX], ry = gp[G_RY], rz = gp[G_RZ];
  const float sw = gp[G_SW], r = gp[G_R], dsw_dr = gp[G_DSW];
  const float4 dR = *(const float4 *)(dRt + 4 * (size_t)p);
  const float4 ga = *(const float4 *)(gr + 4 * (size_t)p);
  // R~ = (s, s rhat)
  const float ds = gs[p] + dR.x + dR.y * rx + dR.z * ry + dR.w * rz;
  float drx = ga.x + s * dR.y;
  float dry = ga.y + s * dR.z;
  float drz = ga.z + s * dR.w;
  // s = sw / r
  const float inv_r = 1.0f / r;
  const float dsw = gw[p] + ds * inv_r;
  const float dr = -ds * sw * inv_r * inv_r + dsw * dsw_dr;
  // rhat = d / r: tangential projection
  const float proj = drx * rx + dry * ry + drz * rz;
  float4 out;
  out.x = dr * rx + (drx - proj * rx) * inv_r;
  out.y = dr * ry + (dry - proj * ry) * inv_r;
  out.z = dr * rz + (drz - proj * rz) * inv_r;
  out.w = 0.f;
  *(float4 *)(gout + 4 * (size_t)p) = out;
}

__device__ __forceinline__ int find_slot(const int *__restrict__ row, int n, int key) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = row[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// one wavefront per atom (locals and ghosts)
__global__ __launch_bounds__(256) void k_forces(const double *__restrict__ x, CellGrid grid,
                                                int nloc, int nall, int sel,
                                                const int *__restrict__ nlist,
                                                const int *__restrict__ nnei,
                                                const int *__restrict__ pair_off,
                                                const float *__restrict__ g,
                                                const double *__restrict__ wgt, double sign,
                                                double *__restrict__ forces,
                                                double *__restrict__ vir_part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + wave;
  if (k >= nall) return;
  const int nk = nnei[k];
  const int *row = nlist + (size_t)k * sel;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0;
  double v[9];
  for (int c = 0; c < 9; ++c) v[c] = 0.0;
  const bool local = k < nloc;
  const int base = local ? pair_off[k] : 0;
  const double wk = (local && wgt) ? wgt[k] : 1.0;
  for (int s = lane; s < nk; s += kWave) {
    const int j = row[s];
    if (local) {
      const float4 gk = *(const float4 *)(g + 4 * (size_t)(base + s));
      const double gx = wk * gk.x, gy = wk * gk.y, gz = wk * gk.z;
      f0 += gx;
      f1 += gy;
      f2 += gz;
      double d[3];
      pair_vec(x, k, j, grid, d);
      v[0] -= d[0] * gx; v[1] -= d[0] * gy; v[2] -= d[0] * gz;
      v[3] -= d[1] * gx; v[4] -= d[1] * gy; v[5] -= d[1] * gz;
      v[6] -= d[2] * gx; v[7] -= d[2] * gy; v[8] -= d[2] * gz;
    }
    if (j < nloc) {
      const int t = find_slot(nlist + (size_t)j * sel, nnei[j], k);
      if (t >= 0) {
        const float4 gj = *(const float4 *)(g + 4 * (size_t)(pair_off[j] + t));
        const double wj = wgt ? wgt[j] : 1.0;
        f0 -= wj * gj.x;
        f1 -= wj * gj.y;
        f2 -= wj * gj.z;
      }
    }
  }
  f0 = wave_sum(f0);
  f1 = wave_sum(f1);
  f2 = wave_sum(f2);
  if (local)
    for (int c = 0; c < 9; ++c) v[c] = wave_sum(v[c]);
  if (lane == 0) {
    forces[3 * (size_t)k + 0] = sign * f0;
    forces[3 * (size_t)k + 1] = sign * f1;
    forces[3 * (size_t)k + 2] = sign * f2;
    if (local)
      for (int c = 0; c < 9; ++c) vir_part[9 * (size_t)k + c] = v[c];
  }
}

// Fixed-order FP64 reductions of the energy and the virial, plus the FP64
// copy of the atomic energies.
__global__ __launch_bounds__(512) void k_reduce(const float *__restrict__ e,
                                                 const double *__restrict__ vir_part, int nloc,
                                                 double *__restrict__ energy,
                                                 double *__restrict__ virial,
                                                 double *__restrict__ atom_energy) {
  // energy == nullptr skips the energy, virial == nullptr the virial
  constexpr int T = 512, W = T / 64;
  __shared__ double red[10][W];
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  double acc[10];
  for (int c = 0; c < 10; ++c) acc[c] = 0.0;
  // four atoms per thread and pass, their loads issued before any is added
  // (one load in flight per thread made the pass a chain of HBM latencies)
  constexpr int U = 4;
  for (int i0 = t; i0 < nloc; i0 += T * U) {
    if (energy) {
      float ev[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + T * u;
        ev[u] = i < nloc ? e[i] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + T * u;
        acc[0] += (double)ev[u];
        if (atom_energy && i < nloc) atom_energy[i] = (double)ev[u];
      }
    }
    if (virial) {
      double vv[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + T * u < nloc ? i0 + T * u : 0;
        const bool ok = i0 + T * u < nloc;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const double v = vir_part[9 * (size_t)i + c];
          vv[u][c] = ok ? v : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[1 + c] += vv[u][c];
    }
  }
  for (int c = 0; c < 10; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (t == 0) {
    double tot[10];
    for (int c = 0; c < 10; ++c) {
      tot[c] = 0.0;
      for (int w = 0; w < W; ++w) tot[c] += red[c][w];
    }
    if (energy) energy[0] = tot[0];
    if (virial)
      for (int c = 0; c < 9; ++c) virial[c] = tot[1 + c];
  }
}

}  // namespace

void launch_energy(const float *z3, const float *t3, int ld, int nfit, const float *w_out,
                   float b_out, const float *ebias, const int32_t *types, int nloc, float *e,
                   float *a3, hipStream_t s) {
  if (nloc <= 0) return;
  hipLaunchKernelGGL(k_energy, dim3((nloc + 3) / 4), dim3(256), 0, s, z3, t3, ld, nfit, w_out,
                     b_out, ebias, types, nloc, e, a3);
}

void launch_env_bwd(const float *geom, const float *gs, const float *dRt, const float *gw,
                    const float *gr, const int *Mptr, int Mmax, float, float *g, hipStream_t s) {
  if (Mmax <= 0) return;
  hipLaunchKernelGGL(k_env_bwd, dim3((Mmax + 255) / 256), dim3(256), 0, s, geom, gs, dRt, gw, gr,
                     Mptr, g);
}

void launch_forces(const double *coords, CellGrid grid, int nloc, int nall, int sel,
                   const int *nlist, const int *nnei, const int *pair_off, const float *g,
                   const double *wgt, double sign, double *forces, double *vir_part,
                   hipStream_t s) {
  if (nall <= 0) return;
  hipLaunchKernelGGL(k_forces, dim3((nall + 3) / 4), dim3(256), 0, s, coords, grid, nloc, nall,
                     sel, nlist, nnei, pair_off, g, wgt, sign, forces, vir_part);
}

void launch_reduce(const float *e, const double *vir_part, int nloc, double *energy,
                   double *virial, double *atom_energy, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(512), 0, s, e, vir_part, nloc, energy, virial,
                     atom_energy);
}

}  // namespace dpa1
