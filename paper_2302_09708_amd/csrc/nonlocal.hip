// nl_project: the gather half of the Kleinman-Bylander term (Sec. 2.1, third bullet).
//
// For every atom J, projector a and orbital v:
//   alpha[v][poff_J + a] = gamma_Ja * dV * sum_{s in S_J} chi_J[s, a] * y_v[S_J[s]]
// The paper does this as one dense product per atom (chi_J^T X[S_J]).  Here a wave64
// owns one atom and kV orbitals: it streams the atom's support indices and chi values
// once, gathers the kV orbitals at those points (kV independent loads in flight per
// step), and reduces across lanes in a fixed order (deterministic, no atomics).
//
// nl_scatter: the other half, out[S_J] += sa * chi_J alpha_J, after hx_apply has written
// the stencil, Veff and Chebyshev terms.  It runs per support point rather than per
// atom: one thread owns a point and kS orbitals, sums the point's entries (every atom
// whose support holds the point, in a fixed order) and updates each orbital once, so
// no two threads touch one output and no atomics are needed.
#include "common.h"

namespace chefsi {

template <typename TC>
__device__ __forceinline__ TC wave_sum(TC v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kNlWaves = 4;  // waves per block (same atom, consecutive orbital groups)
constexpr int kNlV = 4;      // orbitals per wave
constexpr int kNlP = 4;      // projectors per pass

template <typename TI, typename TC>
__global__ __launch_bounds__(256) void nl_project_kernel(NlArgs<TI, TC> a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // the hardware deals consecutive block ids to the 8 XCDs in turn; each XCD takes a
  // contiguous run of logical ids, atom fastest, so atoms with overlapping supports (close
  // in the atom order) read their shared points through one L2
  const int64_t logical = (int64_t)(blockIdx.x % 8) * a.per_xcd + blockIdx.x / 8;
  if (logical >= (int64_t)a.n_atoms * a.ngroups) return;
  const int atom = (int)(logical % a.n_atoms);
  const int64_t v0 = ((logical / a.n_atoms) * kNlWaves + wave) * kNlV;
  if (v0 >= a.ns) return;  // whole wave exits together; no block barrier below
  const int s0 = a.supp_off[atom];
  const int n = a.supp_off[atom + 1] - s0;
  const int npj = a.nproj[atom];
  const TC* chi = a.chi + a.chi_off[atom];
  const int* idx = a.supp_idx + s0;
  const TI* y[kNlV];
  bool vok[kNlV];
#pragma unroll
  for (int u = 0; u < kNlV; ++u) {
    vok[u] = v0 + u < a.ns;
    y[u] = a.y + (vok[u] ? v0 + u : v0) * a.nd;
  }
  for (int a0 = 0; a0 < npj; a0 += kNlP) {
    TC acc[kNlV][kNlP];
#pragma unroll
    for (int u = 0; u < kNlV; ++u)
#pragma unroll
      for (int p = 0; p < kNlP; ++p) acc[u][p] = TC(0);
    for (int s = lane; s < n; s += 64) {
      const int i = idx[s];
      TC c[kNlP];
#pragma unroll
      for (int p = 0; p < kNlP; ++p) c[p] = a0 + p < npj ? chi[(int64_t)(a0 + p) * n + s] : TC(0);
      TC yv[kNlV];
#pragma unroll
      for (int u = 0; u < kNlV; ++u) yv[u] = TC(y[u][i]);
#pragma unroll
      for (int u = 0; u < kNlV; ++u)
#pragma unroll
        for (int p = 0; p < kNlP; ++p) acc[u][p] += c[p] * yv[u];
    }
#pragma unroll
    for (int u = 0; u < kNlV; ++u) {
#pragma unroll
      for (int p = 0; p < kNlP; ++p) {
        if (a0 + p >= npj) continue;
        const TC t = wave_sum(acc[u][p]);
        if (lane == 0 && vok[u]) {
          const int q = a.poff[atom] + a0 + p;
          a.alpha[(v0 + u) * a.np_tot + q] = a.gdv[q] * t;
        }
      }
    }
  }
}

template <typename TI, typename TC>
hipError_t launch_nl_project(const NlArgs<TI, TC>& a, hipStream_t s) {
  if (a.n_atoms <= 0 || a.ns <= 0) return hipSuccess;
  const int per_block = kNlWaves * kNlV;
  NlArgs<TI, TC> b = a;
  b.ngroups = (a.ns + per_block - 1) / per_block;
  const int64_t nb = (int64_t)a.n_atoms * b.ngroups;
  b.per_xcd = (int)((nb + 7) / 8);
  hipLaunchKernelGGL((nl_project_kernel<TI, TC>), dim3((unsigned)(b.per_xcd * 8)), dim3(64 * kNlWaves), 0, s, b);
  return hipGetLastError();
}

constexpr int kS = 8;  // orbitals per scatter thread

// Blocks are dealt to the 8 XCDs in turn; XCD k owns the k-th slab of npb8 point blocks
// and runs it for every orbital group, so the slab's entries stay in that XCD's L2 while
// the groups go by (dealt group by group, every XCD would cycle through all entries).
template <typename TC, typename TO>
__global__ __launch_bounds__(256) void nl_scatter_kernel(NsArgs<TC, TO> a, int npb8, int ngroups) {
  const int xcd = blockIdx.x % 8;
  const int j = blockIdx.x / 8;
  const int group = j / npb8;
  const int pb = xcd * npb8 + j % npb8;
  if (group >= ngroups) return;
  const int p = pb * 256 + threadIdx.x;
  if (p >= a.n_pts) return;
  const int64_t v0 = (int64_t)group * kS;
  const int4 r = a.rec[p];
  const int pt = r.x, e0 = r.y, n = r.z;
  const int nv = (int)min<int64_t>(kS, a.ns - v0);
  const TC* al = a.alpha + v0 * a.np_tot;
  TC sum[kS];
#pragma unroll
  for (int u = 0; u < kS; ++u) sum[u] = TC(0);
  for (int e = e0; e < e0 + n; ++e) {
    const int c = a.col[e];
    const TC w = a.val[e];
#pragma unroll
    for (int u = 0; u < kS; ++u)
      if (u < nv) sum[u] += w * al[(int64_t)u * a.np_tot + c];
  }
#pragma unroll
  for (int u = 0; u < kS; ++u) {
    if (u >= nv) break;
    TO* o = a.out + (v0 + u) * a.nd + pt;
    *o = TO(TC(*o) + a.sa * sum[u]);
  }
}

template <typename TC, typename TO>
hipError_t launch_nl_scatter(const NsArgs<TC, TO>& a, hipStream_t s) {
  if (a.n_pts <= 0 || a.ns <= 0) return hipSuccess;
  const int npb = (a.n_pts + 255) / 256;
  const int npb8 = (npb + 7) / 8;
  const int ngroups = (a.ns + kS - 1) / kS;
  hipLaunchKernelGGL((nl_scatter_kernel<TC, TO>), dim3((unsigned)(8 * npb8 * ngroups)), dim3(256), 0, s, a, npb8,
                     ngroups);
  return hipGetLastError();
}

// Orbitals per group: a group's final values of the region's points sit in LDS
// (kBandMaxPts * G * sizeof(TC): 32 KB in FP64, 16 KB in FP32) beside the staged
// coefficients and the entry tables (80 KB in all in FP64: two blocks share a CU).  Eight
// orbitals per group in FP32 too: measured against 16 and 4 (120^3, Ns 7200: 592 vs 609
// and 709 ms per step; 72^3 mixed: 7.5 vs 7.9 and 8.3 ms).
template <typename TC>
constexpr int band_g() { return 8; }

// One block per (region, run of orbital groups), one thread per point.  The region's
// entry tables go to LDS once; then, group by group, the point values and the staged
// coefficients of the next group are fetched into registers while the current group is
// scattered and gathered, so the block streams its orbitals with one barrier pair per
// group.  Blocks are dealt to the 8 XCDs in turn, each XCD taking a contiguous run of
// logical ids (region-major, run of groups fastest).
template <typename TY, typename TC, bool SCATTER>
__global__ __launch_bounds__(kBandThreads) void nl_band_kernel(NbArgs<TY, TC> a, int gather) {
  constexpr int G = band_g<TC>();
  constexpr int AJ = (kBandMaxSlots * G + kBandThreads - 1) / kBandThreads;  // staged coefficients per thread
  __shared__ TC ys[kBandMaxPts * G];
  __shared__ TC as[kBandMaxSlots * G];
  __shared__ TC echi[kBandMaxEnt];
  __shared__ TC gchi[kBandMaxEnt];
  __shared__ unsigned short els[kBandMaxEnt];
  __shared__ unsigned short gloc[kBandMaxEnt];
  __shared__ int sent[kBandMaxSlots + 1];
  __shared__ int sq[kBandMaxSlots];
  const int64_t logical = (int64_t)(blockIdx.x % 8) * a.per_xcd + (a.per_xcd - 1 - blockIdx.x / 8);
  if (logical >= (int64_t)a.nreg * a.nchunks) return;
  const int reg = (int)(logical % a.nreg);
  const int g0 = (int)(logical / a.nreg) * a.gpc;
  const int g1 = min(a.ngroups, g0 + a.gpc);
  if (g0 >= g1) return;
  const int tid = threadIdx.x;
  const int p0 = a.reg_pt[reg], np = a.reg_pt[reg + 1] - p0;
  const int s0 = a.reg_slot[reg], nslot = a.reg_slot[reg + 1] - s0;
  // the region's tables
  const int eb = a.pt_ent[p0];
  if (SCATTER) {
    const int ne = a.pt_ent[p0 + np] - eb;
    for (int e = tid; e < ne; e += kBandThreads) {
      echi[e] = a.ent_chi[eb + e];
      els[e] = (unsigned short)a.ent_ls[eb + e];
    }
  }
  const int gb = a.slot_ent[s0];
  if (gather) {
    const int ne = a.slot_ent[s0 + nslot] - gb;
    for (int e = tid; e < ne; e += kBandThreads) {
      gchi[e] = a.gent_chi[gb + e];
      gloc[e] = (unsigned short)a.gent_loc[gb + e];
    }
  }
  for (int sl = tid; sl <= nslot; sl += kBandThreads) sent[sl] = a.slot_ent[s0 + sl] - gb;
  for (int sl = tid; sl < nslot; sl += kBandThreads) sq[sl] = a.slot_q[s0 + sl];
  const bool own = tid < np;
  int64_t pi = 0;
  int e0 = 0, e1 = 0;
  if (own) {
    pi = a.pt_idx[p0 + tid];
    e0 = a.pt_ent[p0 + tid] - eb;
    e1 = a.pt_ent[p0 + tid + 1] - eb;
  }
  const int nitem = nslot * G;
  auto load_y = [&](int g, TC (&y)[G]) {
    const int v0 = g * G;
#pragma unroll
    for (int u = 0; u < G; ++u) y[u] = own && v0 + u < a.ns ? TC(a.y[(int64_t)(v0 + u) * a.nd + pi]) : TC(0);
  };
  auto load_alpha = [&](int g, TC (&an)[AJ]) {
    const int v0 = g * G;
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const int it = tid + j * kBandThreads, ls = it / G, u = it % G;
      an[j] = it < nitem && v0 + u < a.ns ? a.alpha[(int64_t)sq[ls] * a.ns + v0 + u] : TC(0);
    }
  };
  auto stage_alpha = [&](const TC (&an)[AJ]) {
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const int it = tid + j * kBandThreads;
      if (it < nitem) as[it] = an[j];
    }
  };
  __syncthreads();  // slot columns staged
  TC yc[G], yn[G], an[AJ];
  load_y(g0, yc);
  if (SCATTER) {
    load_alpha(g0, an);
    stage_alpha(an);
  }
  __syncthreads();
  for (int g = g0; g < g1; ++g) {
    const int v0 = g * G, nv = min(G, a.ns - v0);
    const bool more = g + 1 < g1;
    if (more) {
      load_y(g + 1, yn);
      if (SCATTER) load_alpha(g + 1, an);
    }
    if (own) {
      TC y[G];
#pragma unroll
      for (int u = 0; u < G; ++u) y[u] = yc[u];
      if (SCATTER) {
        TC t[G];
#pragma unroll
        for (int u = 0; u < G; ++u) t[u] = TC(0);
        for (int e = e0; e < e1; ++e) {
          const TC c = echi[e];
          const TC* al = as + els[e] * G;
#pragma unroll
          for (int u = 0; u < G; ++u) t[u] += c * al[u];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
          if (u >= nv) break;
          y[u] += a.sa * t[u];
          a.y[(int64_t)(v0 + u) * a.nd + pi] = TY(y[u]);
          y[u] = TC(TY(y[u]));  // the gather reads the stored value
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) ys[tid * G + u] = y[u];
    }
    __syncthreads();  // ys complete; the staged coefficients are no longer read
    if (SCATTER && more) stage_alpha(an);
    if (gather) {
      // slot partials: one thread per (slot, orbital), the slot's entries in index order
      for (int it = tid; it < nitem; it += kBandThreads) {
        const int sl = it / G, u = it % G;
        if (u >= nv) continue;
        // four running sums over entries e = 4 m + c (independent LDS chains), added in a
        // fixed order
        TC s4[4] = {TC(0), TC(0), TC(0), TC(0)};
        const int eb0 = sent[sl], ee = sent[sl + 1];
        int e = eb0;
        for (; e + 4 <= ee; e += 4) {
#pragma unroll
          for (int c = 0; c < 4; ++c) s4[c] += gchi[e + c] * ys[gloc[e + c] * G + u];
        }
        for (int c = 0; e < ee; ++e, ++c) s4[c] += gchi[e] * ys[gloc[e] * G + u];
        a.partial[(int64_t)(s0 + sl) * a.ns + v0 + u] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
      }
    }
    __syncthreads();  // ys free, next coefficients staged
#pragma unroll
    for (int u = 0; u < G; ++u) yc[u] = yn[u];
  }
}

template <typename TY, typename TC>
hipError_t launch_nl_band(const NbArgs<TY, TC>& a0, bool scatter, bool gather, hipStream_t s) {
  if (a0.nreg <= 0 || a0.ns <= 0) return hipSuccess;
  NbArgs<TY, TC> a = a0;
  constexpr int G = band_g<TC>();
  a.ngroups = (a.ns + G - 1) / G;
  // runs of groups: about 4096 blocks in all (16 per CU at two resident per CU), each run
  // as long as that allows (the tables are staged once per run)
  const int want = (int)std::min<int64_t>(a.ngroups, std::max<int64_t>(1, (4096 + a.nreg - 1) / a.nreg));
  a.gpc = (a.ngroups + want - 1) / want;
  a.nchunks = (a.ngroups + a.gpc - 1) / a.gpc;
  const int64_t nb = (int64_t)a.nreg * a.nchunks;
  a.per_xcd = (int)((nb + 7) / 8);
  const dim3 grid((unsigned)(a.per_xcd * 8));
  if (scatter)
    hipLaunchKernelGGL((nl_band_kernel<TY, TC, true>), grid, dim3(kBandThreads), 0, s, a, gather ? 1 : 0);
  else
    hipLaunchKernelGGL((nl_band_kernel<TY, TC, false>), grid, dim3(kBandThreads), 0, s, a, 1);
  return hipGetLastError();
}

// alpha[q][v] = gdv[q] * sum over the slots of q (region order) of partial[slot][v].
template <typename TC>
__global__ __launch_bounds__(256) void nl_band_reduce_kernel(const TC* __restrict__ partial,
                                                             const int* __restrict__ q_slot_ptr,
                                                             const int* __restrict__ q_slot,
                                                             const TC* __restrict__ gdv, int np_tot, int ns,
                                                             TC* __restrict__ alpha) {
  const int q = blockIdx.y;
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (q >= np_tot || v >= ns) return;
  TC sum = TC(0);
  for (int k = q_slot_ptr[q]; k < q_slot_ptr[q + 1]; ++k) sum += partial[(int64_t)q_slot[k] * ns + v];
  alpha[(int64_t)q * ns + v] = gdv[q] * sum;
}

template <typename TC>
hipError_t launch_nl_band_reduce(const TC* partial, const int* q_slot_ptr, const int* q_slot, const TC* gdv,
                                 int np_tot, int ns, TC* alpha, hipStream_t s) {
  if (np_tot <= 0 || ns <= 0) return hipSuccess;
  const dim3 grid((unsigned)((ns + 255) / 256), (unsigned)np_tot);
  hipLaunchKernelGGL(nl_band_reduce_kernel<TC>, grid, dim3(256), 0, s, partial, q_slot_ptr, q_slot, gdv, np_tot, ns,
                     alpha);
  return hipGetLastError();
}

template hipError_t launch_nl_band<double, double>(const NbArgs<double, double>&, bool, bool, hipStream_t);
template hipError_t launch_nl_band<float, float>(const NbArgs<float, float>&, bool, bool, hipStream_t);
template hipError_t launch_nl_band<float, double>(const NbArgs<float, double>&, bool, bool, hipStream_t);
template hipError_t launch_nl_band_reduce<double>(const double*, const int*, const int*, const double*, int, int,
                                                  double*, hipStream_t);
template hipError_t launch_nl_band_reduce<float>(const float*, const int*, const int*, const float*, int, int,
                                                 float*, hipStream_t);

template hipError_t launch_nl_scatter<double, double>(const NsArgs<double, double>&, hipStream_t);
template hipError_t launch_nl_scatter<float, float>(const NsArgs<float, float>&, hipStream_t);

template hipError_t launch_nl_project<double, double>(const NlArgs<double, double>&, hipStream_t);
template hipError_t launch_nl_project<float, float>(const NlArgs<float, float>&, hipStream_t);
template hipError_t launch_nl_project<float, double>(const NlArgs<float, double>&, hipStream_t);

}  // namespace chefsi
