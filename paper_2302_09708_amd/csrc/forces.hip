// Nonlocal Hellmann-Feynman forces (Sec. 2: the filter's stencil and projector routines
// reused for the force: the gradient operator on the orbitals, then the nonlocal
// projectors on the result).  With a = dV chi^T psi and b_d = dV chi^T (d psi / dx_d)
// from the projector gather (nl_project with dV in place of gamma dV),
//
//   F_J,d = -2 sum_n g_n sum_a gamma_Ja a_Ja,n b_d,Ja,n .
//
// grad_kernel: the central FD first derivative of order 2r along one direction, one
// thread per (point, orbital), periodic wrap or zero ghosts; FP64 output.
// force_kernel: one thread per atom, fixed summation order (bitwise reproducible).
#include "common.h"

namespace chefsi {

namespace {

template <typename TV>
__global__ __launch_bounds__(256) void grad_kernel(GradArgs<TV> a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.nd) return;
  const int64_t v = blockIdx.y;
  const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((int64_t)a.nx * a.ny));
  const int c = a.dir == 0 ? x : (a.dir == 1 ? y : z);
  const int n = a.dir == 0 ? a.nx : (a.dir == 1 ? a.ny : a.nz);
  const int64_t stride = a.dir == 0 ? 1 : (a.dir == 1 ? (int64_t)a.nx : (int64_t)a.nx * a.ny);
  const TV* col = a.x + v * a.nd;
  const int64_t base = i - (int64_t)c * stride;
  double g = 0.0;
  for (int p = 1; p <= a.r; ++p) {
    int cp = c + p, cm = c - p;
    double fp, fm;
    if (a.periodic) {
      cp %= n;
      cm = ((cm % n) + n) % n;
      fp = double(col[base + cp * stride]);
      fm = double(col[base + cm * stride]);
    } else {
      fp = cp < n ? double(col[base + cp * stride]) : 0.0;
      fm = cm >= 0 ? double(col[base + cm * stride]) : 0.0;
    }
    g += a.c[p] * (fp - fm);
  }
  a.out[v * a.nd + i] = g * a.inv_h;
}

__global__ __launch_bounds__(256) void force_kernel(ForceArgs a) {
  const int J = blockIdx.x * 256 + threadIdx.x;
  if (J >= a.n_atoms) return;
  double acc = 0.0;
  for (int k = 0; k < a.nproj[J]; ++k) {
    const int q = a.poff[J] + k;
    const double gam = a.gdv[q] / a.dv;
    double s = 0.0;
    for (int v = 0; v < a.ns; ++v) {
      const int64_t e = (int64_t)v * a.np_tot + q;
      s += a.occ[v] * a.alpha[e] * a.beta[e];
    }
    acc += gam * s;
  }
  a.forces[(int64_t)J * 3 + a.dir] = -2.0 * acc;
}

}  // namespace

template <typename TV>
hipError_t launch_grad(const GradArgs<TV>& a, int ns, hipStream_t s) {
  if (ns <= 0 || a.nd <= 0) return hipSuccess;
  hipLaunchKernelGGL((grad_kernel<TV>), dim3((unsigned)((a.nd + 255) / 256), (unsigned)ns), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_forces(const ForceArgs& a, hipStream_t s) {
  if (a.n_atoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(force_kernel, dim3((unsigned)((a.n_atoms + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_grad<double>(const GradArgs<double>&, int, hipStream_t);
template hipError_t launch_grad<float>(const GradArgs<float>&, int, hipStream_t);

}  // namespace chefsi
