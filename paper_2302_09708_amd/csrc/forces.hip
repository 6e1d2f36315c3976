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

// FD gradient of orbital column `col` at point i along `dir` (the same stencil as grad_kernel).
template <typename TV>
__device__ __forceinline__ double fd_grad(const StressArgs<TV>& a, const TV* col, int64_t i, int x, int y, int z,
                                          int dir) {
  const int c = dir == 0 ? x : (dir == 1 ? y : z);
  const int n = dir == 0 ? a.nx : (dir == 1 ? a.ny : a.nz);
  const int64_t stride = dir == 0 ? 1 : (dir == 1 ? (int64_t)a.nx : (int64_t)a.nx * a.ny);
  const int64_t base = i - (int64_t)c * stride;
  double g = 0.0;
  for (int p = 1; p <= a.r; ++p) {
    int cp = c + p, cm = c - p;
    double fp, fm;
    if (a.periodic[dir]) {
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
  return g * a.inv_h[dir];
}

// Six sums sum_v occ[v] sum_i g_a g_b (ab = xx, yy, zz, xy, xz, yz) over a fixed grid-stride
// walk of (orbital, point); per-block partials, reduced by stress_sum_kernel.
template <typename TV>
__global__ __launch_bounds__(256) void stress_partial_kernel(StressArgs<TV> a) {
  __shared__ double red[6][256];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t total = a.nd * a.ns;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t v = e / a.nd, i = e % a.nd;
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((int64_t)a.nx * a.ny));
    const TV* col = a.x + v * a.nd;
    const double gx = fd_grad(a, col, i, x, y, z, 0);
    const double gy = fd_grad(a, col, i, x, y, z, 1);
    const double gz = fd_grad(a, col, i, x, y, z, 2);
    const double w = a.occ[v];
    acc[0] += w * gx * gx;
    acc[1] += w * gy * gy;
    acc[2] += w * gz * gz;
    acc[3] += w * gx * gy;
    acc[4] += w * gx * gz;
    acc[5] += w * gy * gz;
  }
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 6) a.partial[(int64_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void stress_sum_kernel(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ out) {
  if (threadIdx.x >= 6) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * 6 + threadIdx.x];
  out[threadIdx.x] = s;
}

// out[b * nchi + e] = chi[e] * disp[3 s + b], b = 0, 1, 2, for every projector value e of
// atom J (block J) at its support point s: the projectors weighted by the components of the
// displacement of the point from the atom, for the nonlocal stress's strain derivative.
__global__ __launch_bounds__(256) void chi_disp_kernel(ChiDispArgs a) {
  const int J = blockIdx.x;
  const int s0 = a.supp_off[J], nj = a.supp_off[J + 1] - s0;
  const int64_t c0 = a.chi_off[J];
  const int nv = nj * a.nproj[J];
  for (int e = threadIdx.x; e < nv; e += 256) {
    const int s = e % nj;
    const double v = a.chi[c0 + e];
#pragma unroll
    for (int b = 0; b < 3; ++b) a.out[(int64_t)b * a.nchi + c0 + e] = v * a.disp[3 * (int64_t)(s0 + s) + b];
  }
}

}  // namespace

hipError_t launch_chi_disp(const ChiDispArgs& a, hipStream_t s) {
  if (a.n_atoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(chi_disp_kernel, dim3((unsigned)a.n_atoms), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename TV>
hipError_t launch_stress_sums(const StressArgs<TV>& a, hipStream_t s) {
  hipLaunchKernelGGL((stress_partial_kernel<TV>), dim3(kVecBlocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(stress_sum_kernel, dim3(1), dim3(64), 0, s, a.partial, kVecBlocks, a.out);
  return hipGetLastError();
}

template hipError_t launch_stress_sums<double>(const StressArgs<double>&, hipStream_t);
template hipError_t launch_stress_sums<float>(const StressArgs<float>&, hipStream_t);

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
