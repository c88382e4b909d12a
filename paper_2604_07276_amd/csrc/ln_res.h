// Row epilogue of an attention layer's output projection (Sec. II-B,
// DPA-1): G_out = G_in + gamma * LN(acc + b) + beta, with LN the layer norm
// over the Nreal real columns (mean, then the mean square of the centred
// values, eps inside the square root), storing the normalised row xhat and
// 1/std for the adjoint.
//
// acc holds the product of one 16-row tile in the matrix-core output layout
// of the row-batched GEMMs: lane l has row l % 16 and columns
// 16 nt + 4 (l / 16) + {0..3}.  Used by the projection GEMM and by the
// attention forward kernel that applies the projection itself, so both give
// the same bits.
#ifndef DPA1_LN_RES_H
#define DPA1_LN_RES_H

#include <hip/hip_runtime.h>

#include <cstddef>

namespace dpa1 {
namespace lnres {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float row_sum16(float v) {
  // sum over the four lane groups that share (lane % 16)
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// One 16-row tile.  cs: bias, gamma and beta over CW staged columns
// (cs[0..CW), cs[CW..2CW), cs[2CW..3CW)); ntt: column tiles that exist;
// ok: this lane's row is a real row (it is then stored at rb = row * ld);
// gi: the residual row G_in, loaded by the caller.
template <int NT>
__device__ __forceinline__ void apply_tile(floatx4 (&acc)[NT], const floatx4 (&gi)[NT], int g,
                                           int ntt, int Nreal, float eps, const float *cs,
                                           int CW, bool ok, int row, size_t rb, float *gout,
                                           float *xhat, float *rstd) {
  const float invn = 1.0f / (float)Nreal;
  float s1 = 0.f;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const floatx4 b = *(const floatx4 *)(cs + nt * 16 + 4 * g);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = nt * 16 + 4 * g + v;
      const bool in = nt < ntt && n < Nreal;
      acc[nt][v] = in ? acc[nt][v] + b[v] : 0.f;
      s1 += acc[nt][v];
    }
  }
  const float mean = row_sum16(s1) * invn;
  float s2 = 0.f;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = nt * 16 + 4 * g + v;
      const float c = acc[nt][v] - mean;
      s2 += (nt < ntt && n < Nreal) ? c * c : 0.f;
    }
  }
  const float var = row_sum16(s2) * invn;
  const float rs = 1.0f / sqrtf(var + eps);
  if (!ok) return;
  if (g == 0) rstd[row] = rs;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    if (nt >= ntt) continue;
    const int n0 = nt * 16 + 4 * g;
    const floatx4 gm = *(const floatx4 *)(cs + CW + n0);
    const floatx4 bt = *(const floatx4 *)(cs + 2 * CW + n0);
    floatx4 go, xh;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bool in = n0 + v < Nreal;
      const float x = (acc[nt][v] - mean) * rs;
      xh[v] = in ? x : 0.f;
      go[v] = in ? gi[nt][v] + gm[v] * x + bt[v] : 0.f;
    }
    *(floatx4 *)(gout + rb + n0) = go;
    *(floatx4 *)(xhat + rb + n0) = xh;
  }
}

}  // namespace lnres
}  // namespace dpa1

#endif  // DPA1_LN_RES_H
