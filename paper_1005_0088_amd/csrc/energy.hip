// Energy density matrix on the pattern, pole form of Eq. (10):
//   e = M1 + kappa M0 + sum_p Im(-(4i/beta) G(alpha_p) R_p alpha_p)
//     = M1 + kappa M0 + sum_p Re(c_p G(alpha_p)),   c_p = w_p alpha_p,
// with w_p = -(4/beta) R_p, kappa = (4/beta) sum_p R_p (Eq. (11)) and M0, M1
// the zeroth and first moments of G (S^-1 and S^-1 H S^-1).  The selected
// G(alpha_p) are the ones the density matrix of Eq. (8) sums, read from the
// same pattern slots of the pole-batched panels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ndrho {

// acc_e = m1 + kappa m0 over the pattern (sorted order)
__global__ __launch_bounds__(256) void k_init_edm(const double* __restrict__ m1, const double* __restrict__ m0,
                                                  double kappa, int64_t count, double* __restrict__ acc_e) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k < count) acc_e[k] = m1[k] + kappa * m0[k];
}

// acc_e += sum_p Re(c_p G_p) at every pattern slot, poles in their order;
// with several structures in one plan, slot k takes the weights of its
// structure ssid[k], cstride entries apart (ssid NULL: one structure)
__global__ __launch_bounds__(256) void k_accum_edm(const int64_t* __restrict__ slot, int64_t count,
                                                   const double2* __restrict__ panel, int64_t ps,
                                                   const double2* __restrict__ cw, int npoles,
                                                   const int32_t* __restrict__ ssid, int64_t cstride,
                                                   double* __restrict__ acc_e) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= count) return;
  const double2* g = panel + slot[k];
  if (ssid) cw += int64_t(ssid[k]) * cstride;
  double v = acc_e[k];
  for (int p = 0; p < npoles; ++p) {
    const double2 x = g[int64_t(p) * ps];
    const double2 c = cw[p];
    v += c.x * x.x - c.y * x.y;
  }
  acc_e[k] = v;
}

static inline unsigned edm_blocks(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

hipError_t launch_init_edm(const double* m1, const double* m0, double kappa, int64_t count, double* acc_e,
                           hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_edm, dim3(edm_blocks(count)), dim3(256), 0, st, m1, m0, kappa, count, acc_e);
  return hipGetLastError();
}

hipError_t launch_accum_edm(const int64_t* slot, int64_t count, const double2* panel, int64_t ps,
                            const double2* cw, int npoles, const int32_t* ssid, int64_t cstride, double* acc_e,
                            hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_accum_edm, dim3(edm_blocks(count)), dim3(256), 0, st, slot, count, panel, ps, cw, npoles,
                     ssid, cstride, acc_e);
  return hipGetLastError();
}

}  // namespace ndrho
