// Traces Tr(G(alpha_p) S) = sum_ij G_ij S_ji of the selected Green functions
// over the pattern (S symmetric: S_ji = S_ij), one per pole of a batch.  They
// give the density of states of the retarded Green function,
// -(2/pi) Im Tr(G(E + i eta) S) (Sec. II C 3, Eq. (42)), used by the
// chemical-potential search.  Partial sums per workgroup; the host adds them
// (a fixed order, so the result does not depend on scheduling).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ndrho {

// grid (nblk, npoles); partial[p * nblk + b] = sum over the slots of the
// grid-stride range of block b of G_p[slot[k]] * s[entry[k]]
__global__ __launch_bounds__(256) void k_trace_gs(const int64_t* __restrict__ slot, const int32_t* __restrict__ entry,
                                                  int64_t count, const double2* __restrict__ panel, int64_t ps,
                                                  const double* __restrict__ s, double2* __restrict__ partial) {
  __shared__ double red[2][256];
  const int p = blockIdx.y;
  const double2* g = panel + int64_t(p) * ps;
  double re = 0.0, im = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < count; k += int64_t(gridDim.x) * 256) {
    const double sv = s[entry[k]];
    const double2 x = g[slot[k]];
    re += x.x * sv;
    im += x.y * sv;
  }
  red[0][threadIdx.x] = re;
  red[1][threadIdx.x] = im;
  __syncthreads();
  for (unsigned h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[int64_t(p) * gridDim.x + blockIdx.x] = make_double2(red[0][0], red[1][0]);
}

hipError_t launch_trace_gs(const int64_t* slot, const int32_t* entry, int64_t count, const double2* panel, int64_t ps,
                           const double* s, int npoles, int nblk, double2* partial, hipStream_t st) {
  if (npoles < 1 || nblk < 1) return hipSuccess;
  hipLaunchKernelGGL(k_trace_gs, dim3(static_cast<unsigned>(nblk), static_cast<unsigned>(npoles)), dim3(256), 0, st,
                     slot, entry, count, panel, ps, s, partial);
  return hipGetLastError();
}

}  // namespace ndrho
