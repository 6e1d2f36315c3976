// nl_project: the gather half of the Kleinman-Bylander term (Sec. 2.1, third bullet).
//
// For every atom J, projector a and orbital v:
//   alpha[v][poff_J + a] = gamma_Ja * dV * sum_{s in S_J} chi_J[s, a] * y_v[S_J[s]]
// The paper does this as one dense product per atom (chi_J^T X[S_J]); here a
// wave64 owns one (atom, orbital) pair, streams the atom's support once and
// reduces across lanes in a fixed order (deterministic, no atomics).  The
// scatter half, y[S_J] += chi_J alpha_J, is fused into hx_apply.
#include "common.h"

namespace chefsi {

template <typename TC>
__device__ __forceinline__ TC wave_sum(TC v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename TI, typename TC>
__global__ __launch_bounds__(256) void nl_project_kernel(NlArgs<TI, TC> a) {
  constexpr int kWaves = 4;
  constexpr int kP = 4;  // projectors per pass
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int atom = blockIdx.x;
  const int64_t vec = (int64_t)blockIdx.y * kWaves + wave;
  if (vec >= a.ns) return;  // whole wave exits together; no block barrier below
  const int s0 = a.supp_off[atom];
  const int n = a.supp_off[atom + 1] - s0;
  const int npj = a.nproj[atom];
  const TC* chi = a.chi + a.chi_off[atom];
  const int* idx = a.supp_idx + s0;
  const TI* y = a.y + vec * a.nd;
  for (int a0 = 0; a0 < npj; a0 += kP) {
    TC acc[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) acc[p] = TC(0);
    for (int s = lane; s < n; s += 64) {
      const TC v = TC(y[idx[s]]);
#pragma unroll
      for (int p = 0; p < kP; ++p)
        if (a0 + p < npj) acc[p] += chi[(int64_t)(a0 + p) * n + s] * v;
    }
#pragma unroll
    for (int p = 0; p < kP; ++p) {
      if (a0 + p < npj) {
        const TC t = wave_sum(acc[p]);
        if (lane == 0) {
          const int q = a.poff[atom] + a0 + p;
          a.alpha[vec * a.np_tot + q] = a.gdv[q] * t;
        }
      }
    }
  }
}

template <typename TI, typename TC>
hipError_t launch_nl_project(const NlArgs<TI, TC>& a, hipStream_t s) {
  if (a.n_atoms <= 0 || a.ns <= 0) return hipSuccess;
  dim3 grid((unsigned)a.n_atoms, (unsigned)((a.ns + 3) / 4));
  hipLaunchKernelGGL((nl_project_kernel<TI, TC>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_nl_project<double, double>(const NlArgs<double, double>&, hipStream_t);
template hipError_t launch_nl_project<float, float>(const NlArgs<float, float>&, hipStream_t);
template hipError_t launch_nl_project<float, double>(const NlArgs<float, double>&, hipStream_t);

}  // namespace chefsi
