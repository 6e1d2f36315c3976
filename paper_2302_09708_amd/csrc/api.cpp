// Host runtime of libchefsi: handle, validation, workspace plan, CheFSI step orchestration,
// FP64 dense stage (rocSOLVER) and the C-ABI declared in include/chefsi.h.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/chefsi.h"
#include "common.h"

using namespace chefsi;

namespace {

constexpr int kNumProf = 8;
// P_FALLBACK counts mixed steps whose projection and rotation were redone in FP64 (no time)
enum ProfId { P_HX = 0, P_NL = 1, P_GRAM = 2, P_REDUCE = 3, P_ROT = 4, P_EIG = 5, P_COPY = 6, P_FALLBACK = 7 };

// A mixed step whose scaled overlap matrix has a Cholesky pivot below this (relative to its
// unit diagonal, i.e. cond(S Ms S) beyond ~1e4) redoes projection and rotation in FP64:
// the split-bf16 products (~1e-5 relative) cannot resolve the weakest filtered directions,
// and the rotation would amplify their error by the inverse pivot.
constexpr double kMixedMinPivot = 1e-4;

struct Error {
  int status;
  std::string msg;
};

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) throw Error{CHEFSI_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define BLAS_TRY(expr)                                                                         \
  do {                                                                                         \
    rocblas_status s_ = (expr);                                                                \
    if (s_ != rocblas_status_success)                                                          \
      throw Error{CHEFSI_ERR_SOLVER, std::string(#expr) + ": " + rocblas_status_to_string(s_)}; \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Central second-derivative weights of even order 2r (closed form of the
// Lagrange-interpolation stencil); Sec. 2.1 names only the order n0.
std::vector<double> fd_weights(int order) {
  const int r = order / 2;
  std::vector<double> w(r + 1, 0.0);
  long double s = 0.0L;
  for (int p = 1; p <= r; ++p) s += 1.0L / ((long double)p * p);
  w[0] = (double)(-2.0L * s);
  auto fact = [](int n) {
    long double f = 1.0L;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  for (int p = 1; p <= r; ++p) {
    long double num = 2.0L * fact(r) * fact(r);
    long double den = (long double)p * p * fact(r - p) * fact(r + p);
    w[p] = (double)((p % 2 ? 1.0L : -1.0L) * num / den);
  }
  return w;
}

struct EventPair {
  int id;
  hipEvent_t b, e;
};

}  // namespace

// Scratch of chefsi_apply_h_static: the projector coefficients alpha (np_tot x ns of the
// handle's compute type) live in this file-scope device array instead of a caller
// workspace.  Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, never the device memory: its device
// address is looked up once per device (hipGetSymbolAddress, that device current) and
// only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[CHEFSI_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

// device address of `scratch` on the current device (looked up on first use per device)
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) throw Error{CHEFSI_ERR_HIP, "device ordinal out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      throw Error{CHEFSI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}
}  // namespace


struct chefsi_handle {
  int device = 0;
  size_t device_bytes = 0;  // sum of the handle's own device arrays
  int precision = CHEFSI_FP64;
  int n[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  int bc[3] = {0, 0, 0};
  int order = 12, radius = 6;
  int64_t nd = 0;
  int max_ns = 0;
  double dv = 0.0;
  std::vector<double> w;

  // host copies kept for the spectral bounds
  std::vector<double> veff_h;
  int n_atoms = 0;
  int np_tot = 0;
  std::vector<int64_t> supp_ptr_h;
  std::vector<int> supp_idx_h, nproj_h;
  std::vector<double> chi_h, gamma_h;

  // device data
  double* veff64 = nullptr;
  float* veff32 = nullptr;
  int* supp_off = nullptr;
  int* supp_idx = nullptr;
  int64_t* chi_off = nullptr;
  int* nproj = nullptr;
  int* poff = nullptr;
  double* chi64 = nullptr;
  float* chi32 = nullptr;
  double* gdv64 = nullptr;
  float* gdv32 = nullptr;
  // projector entries grouped by (y tile, z plane) of the stencil tiling: one record per touched point
  HxPlan hx_plan;  // tiling for ns = 1 (checked at create; the z chunking depends on ns)
  int4* rec = nullptr;           // scatter records (points with more than four entries)
  int* hx_rec_ptr = nullptr;     // stencil-pass records (points with at most four entries)
  HxRec<double>* hx_rec64 = nullptr;
  HxRec<float>* hx_rec32 = nullptr;
  int* ent_col = nullptr;
  double* ent_val64 = nullptr;
  float* ent_val32 = nullptr;
  // pinned host staging for the small device-to-host reads of every step (Ritz values,
  // dense-stage status, Cholesky pivots): max_ns doubles + 16 status words
  double* pinned = nullptr;
  int n_pts = 0;     // scatter records
  int n_hxrec = 0;   // stencil-pass records
  size_t hx_rec_bytes = 0;   // device bytes of the stencil-pass records
  size_t scatter_bytes = 0;  // device bytes of the scatter records and entries
  // points in at most this many projector entries take their projector term inside the
  // stencil pass (4: the record width), the others in the scatter pass; 0: every term in
  // the band pass (nl_band) instead
  int rec_max = 4;
  // band-pass tables (built while rec_max == 0)
  int nb_reg = 0, nb_pts = 0, nb_slots = 0;
  int* nb_reg_pt = nullptr;
  int* nb_pt_idx = nullptr;
  int* nb_pt_ent = nullptr;
  int* nb_ent_ls = nullptr;
  int* nb_slot_q = nullptr;
  double* nb_ent_chi64 = nullptr;
  float* nb_ent_chi32 = nullptr;
  int* nb_reg_slot = nullptr;
  int* nb_slot_ent = nullptr;
  int* nb_gent_loc = nullptr;
  double* nb_gent_chi64 = nullptr;
  float* nb_gent_chi32 = nullptr;
  int* nb_q_slot_ptr = nullptr;
  int* nb_q_slot = nullptr;
  void* nb_partial = nullptr;  // nb_slots x max_ns values (8 bytes each)
  size_t nb_bytes = 0;

  rocblas_handle blas = nullptr;
  std::map<int, size_t> solver_ws_cache;
  // point-major projector table (host): point i lists pt_col/pt_val[pt_cnt[i] .. pt_cnt[i+1]),
  // kept so the stencil-pass records can be rebuilt for another tiling
  std::vector<int> pt_cnt, pt_col;
  std::vector<double> pt_val;

  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<EventPair> ev_pending;
  double prof_ms[kNumProf] = {0};
  int64_t prof_n[kNumProf] = {0};

  int last_info = 0;
  std::string last_error;
};

namespace {

// FP64 Gram products through rocBLAS as split-K: `splits` K chunks of kc rows as one
// strided-batched dgemm, the tail rows (fewer than splits) as one more dgemm, and the
// partial products summed in a fixed order.  Chunks are no shorter than 2048 rows and
// about 4096 output tiles of 128 x 128 are in flight over all chunks.
// Only the upper triangle of the symmetric product is needed: the columns are cut into
// blocks and block row i is formed against columns [start_i, ns) alone, which skips most
// of the lower triangle's work.
constexpr int kMaxGramBlocks = 8;

struct BlasGram {
  int splits = 1;
  int64_t kc = 0, tail = 0;
  int nparts = 1;
  size_t bytes = 0;
  int nblk = 1;                         // column blocks
  int start[kMaxGramBlocks + 1] = {0};  // block b is columns [start[b], start[b+1])
};

// Column blocks of the upper-triangle Gram (split-K batches of rocBLAS dgemm, measured at
// ns = 600 and 1200): up to ns = 1024, blocks of 128 columns (ns = 600: 2.6 vs 4.2 ms for
// the full product); above, three blocks cut near 0.43 ns and 0.75 ns (ns = 1200 at 512
// and 896: 21.0 vs 28.8 ms); small blocks run too few tiles to pay.
void gram_blocks(int ns, int& nblk, int* start) {
  nblk = 0;
  start[0] = 0;
  if (ns < 256) {
    nblk = 1;
  } else if (ns <= 128 * kMaxGramBlocks) {
    for (int c = 128; c < ns; c += 128) start[++nblk] = c;
    ++nblk;
  } else {
    start[1] = (int)std::lround(0.43 * ns / 128.0) * 128;
    start[2] = (int)std::lround(0.75 * ns / 128.0) * 128;
    nblk = 3;
  }
  start[nblk] = ns;
}

BlasGram plan_blas_gram(int64_t nd, int ns) {
  BlasGram b;
  const int64_t tiles = ((int64_t)(ns + 127) / 128) * ((ns + 127) / 128);
  b.splits = (int)std::max<int64_t>(1, std::min<int64_t>({128, 4096 / tiles, nd / 2048}));
  b.kc = nd / b.splits;
  b.tail = nd - b.kc * b.splits;
  b.nparts = b.splits + (b.tail > 0 ? 1 : 0);
  b.bytes = (size_t)b.nparts * ns * ns * sizeof(double);
  gram_blocks(ns, b.nblk, b.start);
  return b;
}

// FP64 products of the FP32 block of a mixed handle (its FP64 Rayleigh-Ritz pass): the
// block is widened to FP64 one row panel at a time and each panel goes to rocBLAS dgemm.
// A panel is `splits` chunks of kc rows; the Gram partials of chunk q of every panel
// accumulate into partial q in panel order, then the partials are summed in a fixed
// order.  A panel holds at most kPanelBytes and a quarter of the rows, so it fits beside
// the FP32 result in the upper half of the FP64 scratch block.
constexpr int64_t kPanelBytes = (int64_t)512 << 20;

struct PanelPlan {
  int splits = 1;
  int64_t kc = 0, rows = 0;
  size_t part_bytes = 0;   // one set of Gram partials
  size_t panel_bytes = 0;  // one rows x ns FP64 panel
};

PanelPlan plan_panels(int64_t nd, int ns) {
  PanelPlan p;
  const int64_t tiles = ((int64_t)(ns + 127) / 128) * ((ns + 127) / 128);
  const int64_t budget = std::max<int64_t>(1, std::min<int64_t>(kPanelBytes / ((int64_t)ns * 8), nd / 4));
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>({128, 4096 / tiles, budget / 2048}));
  const int64_t kc = std::max<int64_t>(1, budget / splits);
  p.splits = (int)splits;
  p.kc = kc;
  p.rows = splits * kc;
  p.part_bytes = (size_t)splits * ns * ns * sizeof(double);
  p.panel_bytes = (size_t)p.rows * ns * sizeof(double);
  return p;
}

struct WsLayout {
  size_t bufB = 0, alpha = 0, hs = 0, ms = 0, d = 0, e = 0, sc = 0, info = 0, partial = 0, zsplit = 0, panel = 0,
         panel_out = 0, solver = 0, total = 0;
  size_t bufB_bytes = 0, solver_bytes = 0;
  GramPlan gram;
  BlasGram bgram;   // FP64 handles: Gram products of FP64 blocks
  PanelPlan pan;    // mixed handles: FP64 products of the FP32 block
};

// status words in the pinned staging buffer, after max_ns doubles
rocblas_int* pinned_info(chefsi_handle* h) { return reinterpret_cast<rocblas_int*>(h->pinned + h->max_ns); }

size_t elem_bytes(const chefsi_handle* h) { return h->precision == CHEFSI_FP64 ? 8 : 4; }


// Device workspace of the FP64 dense stage (Cholesky, two triangular solves for the
// reduced matrix, symmetric eigensolve, back substitution); the calls run in sequence,
// so the largest single request is enough.
size_t solver_workspace(chefsi_handle* h, int ns) {
  auto it = h->solver_ws_cache.find(ns);
  if (it != h->solver_ws_cache.end()) return it->second;
  const double one = 1.0;
  size_t best = 0, sz = 0;
  auto query = [&](auto&& call) {
    BLAS_TRY(rocblas_start_device_memory_size_query(h->blas));
    call();
    BLAS_TRY(rocblas_stop_device_memory_size_query(h->blas, &sz));
    best = std::max(best, sz);
  };
  query([&] { rocsolver_dpotrf(h->blas, rocblas_fill_upper, ns, nullptr, ns, nullptr); });
  query([&] {
    rocblas_dtrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                  rocblas_diagonal_non_unit, ns, ns, &one, nullptr, ns, nullptr, ns);
  });
  query([&] {
    rocblas_dtrsm(h->blas, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                  rocblas_diagonal_non_unit, ns, ns, &one, nullptr, ns, nullptr, ns);
  });
  query([&] {
    rocblas_dtrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                  rocblas_diagonal_non_unit, ns, ns, &one, nullptr, ns, nullptr, ns);
  });
  query([&] {
    rocsolver_dsyevd(h->blas, rocblas_evect_original, rocblas_fill_upper, ns, nullptr, ns, nullptr, nullptr,
                     nullptr);
  });
  if (h->precision == CHEFSI_FP64) {
    const BlasGram b = plan_blas_gram(h->nd, ns);
    query([&] {
      rocblas_dgemm_strided_batched(h->blas, rocblas_operation_transpose, rocblas_operation_none, ns, ns,
                                    (rocblas_int)b.kc, &one, nullptr, (rocblas_int)h->nd, b.kc, nullptr,
                                    (rocblas_int)h->nd, b.kc, &one, nullptr, ns, (rocblas_stride)ns * ns, b.splits);
    });
  } else {
    const PanelPlan p = plan_panels(h->nd, ns);
    query([&] {
      rocblas_dgemm_strided_batched(h->blas, rocblas_operation_transpose, rocblas_operation_none, ns, ns,
                                    (rocblas_int)p.kc, &one, nullptr, (rocblas_int)p.rows, p.kc, nullptr,
                                    (rocblas_int)h->nd, p.kc, &one, nullptr, ns, (rocblas_stride)ns * ns, p.splits);
    });
    query([&] {
      rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)p.rows, ns, ns, &one,
                    nullptr, (rocblas_int)p.rows, nullptr, ns, &one, nullptr, (rocblas_int)p.rows);
    });
  }
  if ((int64_t)h->nd * ns < ((int64_t)1 << 31))
    query([&] {
      rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)h->nd, ns, ns, &one,
                    nullptr, (rocblas_int)h->nd, nullptr, ns, &one, nullptr, (rocblas_int)h->nd);
    });
  h->solver_ws_cache[ns] = best;
  return best;
}

WsLayout layout(chefsi_handle* h, int ns) {
  WsLayout L;
  size_t off = 0;
  L.bufB = off;
  // mixed handles need an FP64 Nd x ns scratch for the FP64 Rayleigh-Ritz pass: same bytes as FP64 X
  L.bufB_bytes = (size_t)h->nd * ns * 8;
  off += align256(L.bufB_bytes);
  L.alpha = off;
  off += align256((size_t)std::max(1, h->np_tot) * ns * 8);
  L.hs = off;
  off += align256((size_t)ns * ns * 8);
  L.ms = off;
  off += align256((size_t)ns * ns * 8);
  L.d = off;
  off += align256((size_t)ns * 8);
  L.e = off;
  off += align256((size_t)ns * 8);
  L.sc = off;
  off += align256((size_t)ns * 8);
  L.info = off;
  off += 256;
  L.gram = plan_gram(h->nd, ns);
  L.bgram = plan_blas_gram(h->nd, ns);
  L.pan = plan_panels(h->nd, ns);
  L.partial = off;
  off += align256(std::max(L.gram.partial_bytes,
                           h->precision == CHEFSI_FP64 ? L.bgram.bytes : 2 * L.pan.part_bytes));
  L.zsplit = off;
  if (h->precision == CHEFSI_MIXED) off += align256(zsplit_bytes(ns));
  L.panel = off;
  if (h->precision == CHEFSI_MIXED) {
    off += align256(L.pan.panel_bytes);
    // the rotation's FP64 result panel: above the FP32 result in the FP64 scratch block
    // (it fits there unless the grid is tiny), else a region of its own
    L.panel_out = L.bufB + align256((size_t)h->nd * ns * 4);
    if (L.panel_out + L.pan.panel_bytes > L.bufB + align256(L.bufB_bytes)) {
      L.panel_out = off;
      off += align256(L.pan.panel_bytes);
    }
  }
  L.solver = off;
  L.solver_bytes = solver_workspace(h, ns);
  off += align256(std::max<size_t>(L.solver_bytes, 256));
  L.total = off;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---- profiling -------------------------------------------------------------
// HIP events around the launches of one kernel class on the call's stream (any handle type
// with prof_on, ev_pool, ev_pending, prof_ms and prof_n).
template <typename H>
struct ProfScopeT {
  H* h;
  hipStream_t s;
  int id;
  hipEvent_t b = nullptr, e = nullptr;
  ProfScopeT(H* h_, int id_, hipStream_t s_) : h(h_), s(s_), id(id_) {
    if (!h->prof_on) return;
    b = take();
    e = take();
    HIP_TRY(hipEventRecord(b, s));
  }
  hipEvent_t take() {
    if (!h->ev_pool.empty()) {
      hipEvent_t ev = h->ev_pool.back();
      h->ev_pool.pop_back();
      return ev;
    }
    hipEvent_t ev;
    HIP_TRY(hipEventCreate(&ev));
    return ev;
  }
  void done() {
    if (!h->prof_on || b == nullptr) return;
    HIP_TRY(hipEventRecord(e, s));
    h->ev_pending.push_back({id, b, e});
    b = e = nullptr;
  }
  ~ProfScopeT() {
    if (b) h->ev_pool.push_back(b);
    if (e) h->ev_pool.push_back(e);
  }
};
using ProfScope = ProfScopeT<chefsi_handle>;

template <typename H>
void prof_collect(H* h) {
  for (auto& p : h->ev_pending) {
    HIP_TRY(hipEventSynchronize(p.e));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.b, p.e));
    h->prof_ms[p.id] += ms;
    h->prof_n[p.id] += 1;
    h->ev_pool.push_back(p.b);
    h->ev_pool.push_back(p.e);
  }
  h->ev_pending.clear();
}

// ---- argument checks -------------------------------------------------------
void check(bool ok, const char* what) {
  if (!ok) throw Error{CHEFSI_ERR_INVALID_ARG, what};
}

void check_ns(const chefsi_handle* h, int ns) {
  check(ns >= 1 && ns <= h->max_ns, "ns must satisfy 1 <= ns <= max_ns");
  check((int64_t)ns <= h->nd, "ns must not exceed Nd");
}

void check_ws(chefsi_handle* h, int ns, void* ws, size_t ws_bytes, WsLayout& L) {
  L = layout(h, ns);
  if (ws == nullptr || ws_bytes < L.total)
    throw Error{CHEFSI_ERR_WORKSPACE, "workspace smaller than chefsi_workspace_bytes(ns)"};
  check(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
}

void check_bounds(double lo, double cut, double hi) {
  check(std::isfinite(lo) && std::isfinite(cut) && std::isfinite(hi), "spectral bounds must be finite");
  check(lo <= cut && cut < hi, "bounds must satisfy lam_lo <= lam_cut < lam_hi");
}

// ---- kernel wrappers -------------------------------------------------------
template <typename TI, typename TC, typename TO>
HxArgs<TI, TC, TO> hx_args(const chefsi_handle* h, const TI* x, const TO* prev, TO* out, const TC* veff,
                           const TC* alpha) {
  HxArgs<TI, TC, TO> a{};
  a.x = x;
  a.prev = prev;
  a.out = out;
  a.veff = veff;
  a.rec_ptr = h->n_hxrec > 0 ? h->hx_rec_ptr : nullptr;
  if constexpr (sizeof(TC) == 8)
    a.rec = h->hx_rec64;
  else
    a.rec = h->hx_rec32;
  a.alpha = alpha;
  a.np_tot = h->np_tot;
  a.nx = h->n[0];
  a.ny = h->n[1];
  a.nz = h->n[2];
  a.nd = h->nd;
  a.per_x = h->bc[0] == 0;
  a.per_y = h->bc[1] == 0;
  a.per_z = h->bc[2] == 0;
  double sumh = 0.0;
  for (int d = 0; d < 3; ++d) sumh += 1.0 / (h->h[d] * h->h[d]);
  a.c0 = TC(-0.5 * h->w[0] * sumh);
  for (int p = 0; p <= kMaxRadius; ++p) {
    const double wp = p <= h->radius ? h->w[p] : 0.0;
    a.cx[p] = TC(-0.5 * wp / (h->h[0] * h->h[0]));
    a.cy[p] = TC(-0.5 * wp / (h->h[1] * h->h[1]));
    a.cz[p] = TC(-0.5 * wp / (h->h[2] * h->h[2]));
  }
  a.sa = TC(1);
  a.sc = TC(0);
  a.sb = TC(0);
  return a;
}

template <typename TI, typename TC>
NlArgs<TI, TC> nl_args(const chefsi_handle* h, const TI* y, int ns, const TC* chi, const TC* gdv, TC* alpha) {
  NlArgs<TI, TC> a{};
  a.y = y;
  a.nd = h->nd;
  a.ns = ns;
  a.n_atoms = h->n_atoms;
  a.supp_off = h->supp_off;
  a.supp_idx = h->supp_idx;
  a.chi_off = h->chi_off;
  a.nproj = h->nproj;
  a.poff = h->poff;
  a.chi = chi;
  a.gdv = gdv;
  a.alpha = alpha;
  a.np_tot = h->np_tot;
  return a;
}

// out = sa (H x - sc x) + sb prev, with the projector gather for x first.
// out = sa ((H x) - sc x) + sb prev: projector gather (alpha), the stencil + Veff +
// Chebyshev pass, then the projector scatter onto the support points.
// Band-pass arguments for block y (the handle's tables for compute type TC).
template <typename TY, typename TC>
NbArgs<TY, TC> band_args(const chefsi_handle* h, TY* y, int ns, const TC* alpha, double sa) {
  NbArgs<TY, TC> a{};
  a.y = y;
  a.nd = h->nd;
  a.ns = ns;
  a.nreg = h->nb_reg;
  a.reg_pt = h->nb_reg_pt;
  a.pt_idx = h->nb_pt_idx;
  a.pt_ent = h->nb_pt_ent;
  a.ent_ls = h->nb_ent_ls;
  a.slot_q = h->nb_slot_q;
  a.reg_slot = h->nb_reg_slot;
  a.slot_ent = h->nb_slot_ent;
  a.gent_loc = h->nb_gent_loc;
  if constexpr (sizeof(TC) == 8) {
    a.ent_chi = h->nb_ent_chi64;
    a.gent_chi = h->nb_gent_chi64;
  } else {
    a.ent_chi = h->nb_ent_chi32;
    a.gent_chi = h->nb_gent_chi32;
  }
  a.alpha = alpha;
  a.sa = TC(sa);
  a.partial = static_cast<TC*>(h->nb_partial);
  return a;
}

// alpha (projector-major) of block y from the band pass's slot partials
template <typename TY, typename TC>
void band_alpha(chefsi_handle* h, TY* y, int ns, TC* alpha, const TC* gdv, bool scatter, double sa,
                bool want_alpha, hipStream_t s) {
  ProfScope ps(h, P_NL, s);
  HIP_TRY((launch_nl_band<TY, TC>(band_args<TY, TC>(h, y, ns, alpha, sa), scatter, want_alpha, s)));
  if (want_alpha)
    HIP_TRY(launch_nl_band_reduce<TC>(static_cast<const TC*>(h->nb_partial), h->nb_q_slot_ptr, h->nb_q_slot, gdv,
                                      h->np_tot, ns, alpha, s));
  ps.done();
}

// out = sa ((H - sc) x) + sb prev.  The projector term takes one of two routes: stencil-pass
// records plus a scatter pass for the points in more than four entries (the gather nl_project
// first), or, on a handle switched to the band pass, nl_band after a bare stencil pass.  In
// the band route alpha holds projector-major coefficients: alpha_ready says they are already
// those of x (the previous application computed them), want_next asks for those of out.
template <typename TI, typename TC, typename TO>
void apply_fused(chefsi_handle* h, const TI* x, const TO* prev, TO* out, int ns, double sa, double sc, double sb,
                 TC* alpha, hipStream_t s, bool alpha_ready = false, bool want_next = false) {
  const TC* veff;
  const TC* nlv;
  const TC* chi;
  const TC* gdv;
  if constexpr (sizeof(TC) == 8) {
    veff = h->veff64;
    nlv = h->ent_val64;
    chi = h->chi64;
    gdv = h->gdv64;
  } else {
    veff = h->veff32;
    nlv = h->ent_val32;
    chi = h->chi32;
    gdv = h->gdv32;
  }
  const bool band = h->np_tot > 0 && h->rec_max == 0;
  if (band) {
    if (!alpha_ready) band_alpha<TI, TC>(h, const_cast<TI*>(x), ns, alpha, gdv, false, 0.0, true, s);
  } else if (h->np_tot > 0) {
    ProfScope ps(h, P_NL, s);
    HIP_TRY((launch_nl_project<TI, TC>(nl_args<TI, TC>(h, x, ns, chi, gdv, alpha), s)));
    ps.done();
  }
  auto a = hx_args<TI, TC, TO>(h, x, prev, out, veff, alpha);
  a.sa = TC(sa);
  a.sc = TC(sc);
  a.sb = TC(sb);
  {
    ProfScope ps(h, P_HX, s);
    const HxPlan p = plan_hx(h->n[0], h->n[1], h->n[2], ns, h->radius, (int)sizeof(TI), h->hx_plan.py, h->hx_plan.nyg);
    if (!p.ok || p.ty != h->hx_plan.ty)
      throw Error{CHEFSI_ERR_HIP, "stencil tiling differs from the one the projector records were built for"};
    HIP_TRY((launch_hx<TI, TC, TO>(a, p, h->radius, ns, s)));
    ps.done();
  }
  if (band) {
    band_alpha<TO, TC>(h, out, ns, alpha, gdv, true, sa, want_next, s);
  } else if (h->n_pts > 0) {
    NsArgs<TC, TO> n{};
    n.out = out;
    n.nd = h->nd;
    n.ns = ns;
    n.rec = h->rec;
    n.n_pts = h->n_pts;
    n.col = h->ent_col;
    n.val = nlv;
    n.alpha = alpha;
    n.np_tot = h->np_tot;
    n.sa = TC(sa);
    ProfScope ps(h, P_NL, s);
    HIP_TRY((launch_nl_scatter<TC, TO>(n, s)));
    ps.done();
  }
}

// Scaled Chebyshev filter (Alg. 1, Filtering).  Y_0 = X in buffer A; Y_{k+1} overwrites Y_{k-1}.
// Returns the buffer that holds Y_m (A when m is even, B when odd).
// With carry_last, alpha ends as the band-pass coefficients of the returned block.
template <typename T>
T* run_filter(chefsi_handle* h, T* A, T* B, int ns, int m, double lo, double cut, double hi, T* alpha,
              hipStream_t s, bool carry_last = false) {
  const double c = 0.5 * (hi + cut);
  const double e = 0.5 * (hi - cut);
  const double s1 = e / (lo - c);
  double sig = s1;
  // Y_1 = (s1 / e)(H - c) Y_0
  apply_fused<T, T, T>(h, A, nullptr, B, ns, s1 / e, c, 0.0, alpha, s, false, m > 1 || carry_last);
  T* cur = B;
  T* other = A;
  for (int k = 1; k < m; ++k) {
    const double sig_next = 1.0 / (2.0 / s1 - sig);
    apply_fused<T, T, T>(h, cur, other, other, ns, 2.0 * sig_next / e, c, -sig * sig_next, alpha, s, true,
                         k + 1 < m || carry_last);
    std::swap(cur, other);
    sig = sig_next;
  }
  return cur;
}

// Arithmetic of the dense products: FP64 MFMA, or split bf16 (three bf16 MFMAs per
// product, FP32 accumulation) for the FP32 blocks of a mixed handle.
enum class Gemm { F64, BF16X3 };

template <typename TX, typename TY>
hipError_t gram_launch(Gemm g, const TX* X, const TY* Y, int64_t nd, int ns, const GramPlan& p, double* part,
                       hipStream_t s) {
  if constexpr (std::is_same<TX, float>::value && std::is_same<TY, float>::value) {
    if (g == Gemm::BF16X3) return launch_gram_bf16x3(X, Y, nd, ns, p, part, s);
  }
  return launch_gram_f64<TX, TY>(X, Y, nd, ns, p, part, s);
}

// C = X^T Y (upper triangle, mirrored) for FP64 blocks of an FP64 handle: rocBLAS's MFMA
// dgemm over K chunks (a plain GEMM: no fusion to gain), partials summed in a fixed order.
void blas_gram(chefsi_handle* h, const double* X, const double* Y, int ns, const WsLayout& L, void* ws, double* C,
               hipStream_t s) {
  double* part = at<double>(ws, L.partial);
  const BlasGram& b = L.bgram;
  const double one = 1.0, zero = 0.0;
  const rocblas_int ld = (rocblas_int)h->nd;
  {
    ProfScope ps(h, P_GRAM, s);
    BLAS_TRY(rocblas_set_stream(h->blas, s));
    BLAS_TRY(rocblas_set_workspace(h->blas, at<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
    for (int q = 0; q < b.nblk; ++q) {
      // block row q against columns [r0, ns): rows r0 .. r0 + m - 1 of every partial
      const int r0 = b.start[q], m = b.start[q + 1] - r0, n = ns - r0;
      const double* Xq = X + (size_t)r0 * h->nd;
      const double* Yq = Y + (size_t)r0 * h->nd;
      double* Pq = part + r0 + (size_t)r0 * ns;
      BLAS_TRY(rocblas_dgemm_strided_batched(h->blas, rocblas_operation_transpose, rocblas_operation_none, m, n,
                                             (rocblas_int)b.kc, &one, Xq, ld, b.kc, Yq, ld, b.kc, &zero, Pq, ns,
                                             (rocblas_stride)ns * ns, b.splits));
      if (b.tail > 0) {
        const int64_t k0 = b.kc * b.splits;
        BLAS_TRY(rocblas_dgemm(h->blas, rocblas_operation_transpose, rocblas_operation_none, m, n,
                               (rocblas_int)b.tail, &one, Xq + k0, ld, Yq + k0, ld, &zero,
                               Pq + (size_t)b.splits * ns * ns, ns));
      }
    }
    ps.done();
  }
  {
    ProfScope ps(h, P_REDUCE, s);
    HIP_TRY(launch_sum_partials(part, b.nparts, ns, C, s));
    ps.done();
  }
}

// Hs = X^T Y and Ms = X^T X with FP64 arithmetic for the FP32 block X of a mixed handle
// (Y = H X in FP64): each row panel of X is widened once and feeds both rocBLAS products.
// Every FP32 value is exact in FP64, so this is the FP64 product of the stored block.
void panel_gram(chefsi_handle* h, const float* X, const double* Y, int ns, const WsLayout& L, void* ws, double* Hs,
                double* Ms, hipStream_t s) {
  const PanelPlan& p = L.pan;
  double* W = at<double>(ws, L.panel);
  double* partH = at<double>(ws, L.partial);
  double* partM = partH + (size_t)p.splits * ns * ns;
  const double one = 1.0, zero = 0.0;
  const rocblas_int ldw = (rocblas_int)p.rows, ldy = (rocblas_int)h->nd;
  const rocblas_stride pst = (rocblas_stride)ns * ns;
  {
    ProfScope ps(h, P_GRAM, s);
    BLAS_TRY(rocblas_set_stream(h->blas, s));
    BLAS_TRY(rocblas_set_workspace(h->blas, at<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
    for (int64_t r0 = 0; r0 < h->nd; r0 += p.rows) {
      // the first panel is whole (rows <= nd) and sets every partial; later panels add
      const int64_t r = std::min(p.rows, h->nd - r0);
      const double* beta = r0 == 0 ? &zero : &one;
      HIP_TRY(launch_widen_rows(X + r0, h->nd, r, ns, W, p.rows, s));
      const int64_t nfull = r / p.kc, tail = r - nfull * p.kc;
      for (int q = 0; q < L.bgram.nblk; ++q) {
        // upper triangle only: block row q of the product against columns [c0, ns)
        const int c0 = L.bgram.start[q], m = L.bgram.start[q + 1] - c0, n = ns - c0;
        const double* Wq = W + (size_t)c0 * p.rows;
        const double* Yq = Y + r0 + (size_t)c0 * h->nd;
        const size_t co = c0 + (size_t)c0 * ns;
        if (nfull > 0) {
          BLAS_TRY(rocblas_dgemm_strided_batched(h->blas, rocblas_operation_transpose, rocblas_operation_none, m, n,
                                                 (rocblas_int)p.kc, &one, Wq, ldw, p.kc, Yq, ldy, p.kc, beta,
                                                 partH + co, ns, pst, (rocblas_int)nfull));
          BLAS_TRY(rocblas_dgemm_strided_batched(h->blas, rocblas_operation_transpose, rocblas_operation_none, m, n,
                                                 (rocblas_int)p.kc, &one, Wq, ldw, p.kc, Wq, ldw, p.kc, beta,
                                                 partM + co, ns, pst, (rocblas_int)nfull));
        }
        if (tail > 0) {  // only in a last, partial panel: nfull < splits and r0 > 0
          const int64_t k0 = nfull * p.kc;
          BLAS_TRY(rocblas_dgemm(h->blas, rocblas_operation_transpose, rocblas_operation_none, m, n,
                                 (rocblas_int)tail, &one, Wq + k0, ldw, Yq + k0, ldy, &one,
                                 partH + co + nfull * pst, ns));
          BLAS_TRY(rocblas_dgemm(h->blas, rocblas_operation_transpose, rocblas_operation_none, m, n,
                                 (rocblas_int)tail, &one, Wq + k0, ldw, Wq + k0, ldw, &one,
                                 partM + co + nfull * pst, ns));
        }
      }
    }
    ps.done();
  }
  {
    ProfScope ps(h, P_REDUCE, s);
    HIP_TRY(launch_sum_partials(partH, p.splits, ns, Hs, s));
    HIP_TRY(launch_sum_partials(partM, p.splits, ns, Ms, s));
    ps.done();
  }
}

// O = X Z with FP64 arithmetic for the FP32 block X of a mixed handle, rounded once to
// FP32: per row panel, widen, rocBLAS dgemm into the FP64 result panel, narrow into O.
void panel_rotate(chefsi_handle* h, const float* X, const double* Z, float* O, int ns, const WsLayout& L, void* ws,
                  hipStream_t s) {
  ProfScope ps(h, P_ROT, s);
  const PanelPlan& p = L.pan;
  double* W = at<double>(ws, L.panel);
  double* P = at<double>(ws, L.panel_out);
  const double one = 1.0, zero = 0.0;
  BLAS_TRY(rocblas_set_stream(h->blas, s));
  BLAS_TRY(rocblas_set_workspace(h->blas, at<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
  for (int64_t r0 = 0; r0 < h->nd; r0 += p.rows) {
    const int64_t r = std::min(p.rows, h->nd - r0);
    HIP_TRY(launch_widen_rows(X + r0, h->nd, r, ns, W, p.rows, s));
    BLAS_TRY(rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)r, ns, ns, &one, W,
                           (rocblas_int)p.rows, Z, ns, &zero, P, (rocblas_int)p.rows));
    HIP_TRY(launch_narrow_rows(P, p.rows, r, ns, O + r0, h->nd, s));
  }
  ps.done();
}

// Hs = X^T Y, Ms = X^T X (full symmetric, FP64), via split-K partial tiles.
template <typename TX, typename TY>
void gram_pair(chefsi_handle* h, const TX* X, const TY* Y, int ns, const WsLayout& L, void* ws, double* Hs,
               double* Ms, hipStream_t s, Gemm g) {
  if constexpr (std::is_same<TX, double>::value && std::is_same<TY, double>::value) {
    if (h->precision == CHEFSI_FP64) {
      blas_gram(h, X, Y, ns, L, ws, Hs, s);
      blas_gram(h, X, X, ns, L, ws, Ms, s);
      return;
    }
  }
  double* part = at<double>(ws, L.partial);
  {
    ProfScope ps(h, P_GRAM, s);
    HIP_TRY((gram_launch<TX, TY>(g, X, Y, h->nd, ns, L.gram, part, s)));
    ps.done();
  }
  {
    ProfScope ps(h, P_REDUCE, s);
    HIP_TRY(launch_gram_reduce(part, L.gram, ns, Hs, s));
    ps.done();
  }
  {
    ProfScope ps(h, P_GRAM, s);
    HIP_TRY((gram_launch<TX, TX>(g, X, X, h->nd, ns, L.gram, part, s)));
    ps.done();
  }
  {
    ProfScope ps(h, P_REDUCE, s);
    HIP_TRY(launch_gram_reduce(part, L.gram, ns, Ms, s));
    ps.done();
  }
}

// Hs Z = Ms Z D in FP64 on the device (Alg. 1, Diagonalization; Sec. 2.3), as the standard
// reduction of a symmetric-definite pencil after a diagonal scaling S (S_ii = Ms_ii^-1/2):
// S Ms S = U^T U (Cholesky), C = U^-T S Hs S U^-1, C = W D W^T (divide and conquer),
// Z = S U^-1 W.  Z overwrites Hs, U overwrites Ms.  info[0] receives the Cholesky
// status, info[1] the eigensolver status.
// First half: scaling and Cholesky (info[0]); second half: reduction, eigensolve,
// back substitution and back scaling (info[1]).
void dense_factor(chefsi_handle* h, double* Hs, double* Ms, int ns, const WsLayout& L, void* ws, hipStream_t s) {
  ProfScope ps(h, P_EIG, s);
  BLAS_TRY(rocblas_set_stream(h->blas, s));
  BLAS_TRY(rocblas_set_workspace(h->blas, at<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
  rocblas_int* info = at<rocblas_int>(ws, L.info);
  double* sc = at<double>(ws, L.sc);
  HIP_TRY(launch_pencil_scale(Hs, Ms, sc, ns, s));
  BLAS_TRY(rocsolver_dpotrf(h->blas, rocblas_fill_upper, ns, Ms, ns, info));
  ps.done();
}

void dense_solve(chefsi_handle* h, double* Hs, double* Ms, double* D, int ns, const WsLayout& L, void* ws,
                 hipStream_t s) {
  ProfScope ps(h, P_EIG, s);
  const double one = 1.0;
  BLAS_TRY(rocblas_set_stream(h->blas, s));
  BLAS_TRY(rocblas_set_workspace(h->blas, at<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
  rocblas_int* info = at<rocblas_int>(ws, L.info);
  double* sc = at<double>(ws, L.sc);
  BLAS_TRY(rocblas_dtrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                         rocblas_diagonal_non_unit, ns, ns, &one, Ms, ns, Hs, ns));
  BLAS_TRY(rocblas_dtrsm(h->blas, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                         rocblas_diagonal_non_unit, ns, ns, &one, Ms, ns, Hs, ns));
  BLAS_TRY(rocsolver_dsyevd(h->blas, rocblas_evect_original, rocblas_fill_upper, ns, Hs, ns, D,
                            at<double>(ws, L.e), info + 1));
  BLAS_TRY(rocblas_dtrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                         rocblas_diagonal_non_unit, ns, ns, &one, Ms, ns, Hs, ns));
  HIP_TRY(launch_row_scale(Hs, sc, ns, s));
  ps.done();
}

void dense_eig(chefsi_handle* h, double* Hs, double* Ms, double* D, int ns, const WsLayout& L, void* ws,
               hipStream_t s) {
  dense_factor(h, Hs, Ms, ns, L, ws, s);
  dense_solve(h, Hs, Ms, D, ns, L, ws, s);
}

// After dense_factor: true when the Cholesky failed or its smallest pivot U_ii^2 of the
// scaled overlap matrix is below kMixedMinPivot (host round trip; the diagonal of U goes
// through the eigensolver's scratch E, which is free until dense_solve).
bool factor_is_weak(chefsi_handle* h, const double* U, int ns, const WsLayout& L, void* ws, hipStream_t s) {
  double* diag = at<double>(ws, L.e);
  HIP_TRY(launch_copy_diag(U, diag, ns, s));
  double* d = h->pinned;
  rocblas_int* info = pinned_info(h);
  HIP_TRY(hipMemcpyAsync(d, diag, (size_t)ns * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(info, at<rocblas_int>(ws, L.info), sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (info[0] > 0) return true;
  double mn = 1.0;
  for (int i = 0; i < ns; ++i) mn = std::min(mn, d[i] * d[i]);
  return !(mn >= kMixedMinPivot);
}

// Map the two dense-stage status words to a status (the Cholesky failure is reported as
// ns + order of the failing leading minor, the convention of the LAPACK generalized solvers).
void raise_info(chefsi_handle* h, const rocblas_int* info, int ns) {
  if (info[0] > 0) {
    h->last_info = ns + info[0];
    throw Error{CHEFSI_ERR_NOT_POSDEF, "Cholesky of the overlap matrix failed (leading minor " +
                                           std::to_string(info[0]) + ")"};
  }
  if (info[1] > 0) {
    h->last_info = info[1];
    throw Error{CHEFSI_ERR_EIG, "dense eigensolver did not converge"};
  }
}

void check_info(chefsi_handle* h, void* ws, const WsLayout& L, int ns, hipStream_t s) {
  rocblas_int* info = pinned_info(h);
  HIP_TRY(hipMemcpyAsync(info, at<rocblas_int>(ws, L.info), 2 * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  raise_info(h, info, ns);
}

template <typename T>
void copy_block(chefsi_handle* h, T* dst, const T* src, int ns, hipStream_t s) {
  ProfScope ps(h, P_COPY, s);
  HIP_TRY(hipMemcpyAsync(dst, src, (size_t)h->nd * ns * sizeof(T), hipMemcpyDeviceToDevice, s));
  ps.done();
}

template <typename T>
void rotate_into(chefsi_handle* h, const T* X, const double* Z, T* O, int ns, hipStream_t s, Gemm g, void* ws,
                 const WsLayout& L) {
  if constexpr (std::is_same<T, float>::value) {
    if (g == Gemm::F64) {
      panel_rotate(h, X, Z, O, ns, L, ws, s);
      return;
    }
  }
  ProfScope ps(h, P_ROT, s);
  if constexpr (std::is_same<T, float>::value) {
    if (g == Gemm::BF16X3) {
      HIP_TRY(launch_rotate_bf16x3(X, Z, at<void>(ws, L.zsplit), O, h->nd, ns, s));
      ps.done();
      return;
    }
  }
  if constexpr (std::is_same<T, double>::value) {
    // FP64 X Z is a plain GEMM (nd x ns times ns x ns, no fusion): rocBLAS's MFMA kernel for
    // it runs at a higher fraction of the FP64 peak than launch_rotate_f64.  Its 32-bit
    // dimensions bound it to blocks of fewer than 2^31 elements.
    if ((int64_t)h->nd * ns < ((int64_t)1 << 31)) {
      const double one = 1.0, zero = 0.0;
      BLAS_TRY(rocblas_set_stream(h->blas, s));
      BLAS_TRY(rocblas_set_workspace(h->blas, at<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
      BLAS_TRY(rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)h->nd, ns, ns,
                             &one, X, (rocblas_int)h->nd, Z, ns, &zero, O, (rocblas_int)h->nd));
      ps.done();
      return;
    }
  }
  HIP_TRY((launch_rotate_f64<T, T>(X, Z, O, h->nd, ns, s)));
  ps.done();
}

// The dense-product arithmetic of a handle's own steps.
Gemm step_gemm(const chefsi_handle* h) { return h->precision == CHEFSI_MIXED ? Gemm::BF16X3 : Gemm::F64; }

void ritz_to_host(chefsi_handle* h, const double* D, int ns, double* ritz_host, void* ws, const WsLayout& L,
                  hipStream_t s) {
  double* d = h->pinned;
  rocblas_int* info = pinned_info(h);
  HIP_TRY(hipMemcpyAsync(d, D, (size_t)ns * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(info, at<rocblas_int>(ws, L.info), 2 * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  raise_info(h, info, ns);
  for (int i = 0; i < ns; ++i)
    if (!std::isfinite(d[i])) throw Error{CHEFSI_ERR_NONFINITE, "non-finite Ritz value"};
  if (ritz_host) std::memcpy(ritz_host, d, (size_t)ns * 8);
}

// One CheFSI step (Alg. 1) for element type T (double: FP64 handle, float: mixed handle).
template <typename T>
void step_impl(chefsi_handle* h, T* X, int ns, int m, double lo, double cut, double hi, void* ws,
               const WsLayout& L, hipStream_t s, double* ritz_host) {
  T* A = X;
  T* B = at<T>(ws, L.bufB);
  T* alpha = at<T>(ws, L.alpha);
  double* Hs = at<double>(ws, L.hs);
  double* Ms = at<double>(ws, L.ms);
  double* D = at<double>(ws, L.d);
  T* Xf = run_filter<T>(h, A, B, ns, m, lo, cut, hi, alpha, s, true);
  T* Yf = Xf == A ? B : A;
  apply_fused<T, T, T>(h, Xf, nullptr, Yf, ns, 1.0, 0.0, 0.0, alpha, s, true);  // Y~ = H X~
  Gemm g = step_gemm(h);
  gram_pair<T, T>(h, Xf, Yf, ns, L, ws, Hs, Ms, s, g);
  dense_factor(h, Hs, Ms, ns, L, ws, s);
  if (g == Gemm::BF16X3 && factor_is_weak(h, Ms, ns, L, ws, s)) {
    // the filtered block is too ill-conditioned for split-bf16 products: FP64 this step
    g = Gemm::F64;
    h->prof_n[P_FALLBACK] += 1;
    gram_pair<T, T>(h, Xf, Yf, ns, L, ws, Hs, Ms, s, g);
    dense_factor(h, Hs, Ms, ns, L, ws, s);
  }
  dense_solve(h, Hs, Ms, D, ns, L, ws, s);
  rotate_into<T>(h, Xf, Hs, Yf, ns, s, g, ws, L);  // Y~ is dead: X = X~ Z~ goes there
  if (Yf != X) copy_block<T>(h, X, Yf, ns, s);
  ritz_to_host(h, D, ns, ritz_host, ws, L, s);
}

// Optional filter of degree m (storage precision), then a Rayleigh-Ritz pass with FP64
// arithmetic whatever the storage type: H X in FP64 from the stored block, FP64 Gram
// products, the FP64 dense stage and an FP64 rotation rounded once to the storage type.
template <typename T>
void refine_impl(chefsi_handle* h, T* X, int ns, int m, double lo, double cut, double hi, void* ws,
                 const WsLayout& L, hipStream_t s, double* ritz_host) {
  if (m > 0) {
    T* r = run_filter<T>(h, X, at<T>(ws, L.bufB), ns, m, lo, cut, hi, at<T>(ws, L.alpha), s);
    if (r != X) copy_block<T>(h, X, r, ns, s);
  }
  double* HX = at<double>(ws, L.bufB);  // Nd x ns FP64
  double* alpha = at<double>(ws, L.alpha);
  double* Hs = at<double>(ws, L.hs);
  double* Ms = at<double>(ws, L.ms);
  double* D = at<double>(ws, L.d);
  apply_fused<T, double, double>(h, X, nullptr, HX, ns, 1.0, 0.0, 0.0, alpha, s);
  T* B = at<T>(ws, L.bufB);
  if constexpr (std::is_same<T, float>::value) {
    panel_gram(h, X, HX, ns, L, ws, Hs, Ms, s);
    dense_eig(h, Hs, Ms, D, ns, L, ws, s);
    panel_rotate(h, X, Hs, B, ns, L, ws, s);
  } else {
    gram_pair<T, double>(h, X, HX, ns, L, ws, Hs, Ms, s, Gemm::F64);
    dense_eig(h, Hs, Ms, D, ns, L, ws, s);
    rotate_into<T>(h, X, Hs, B, ns, s, Gemm::F64, ws, L);
  }
  copy_block<T>(h, X, B, ns, s);
  ritz_to_host(h, D, ns, ritz_host, ws, L, s);
}

int fail(chefsi_handle* h, const Error& e) {
  if (h) h->last_error = e.msg;
  return e.status;
}

template <typename F>
int guarded(chefsi_handle* h, F&& f) {
  if (h == nullptr) return CHEFSI_ERR_INVALID_ARG;
  try {
    h->last_error.clear();
    h->last_info = 0;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) HIP_TRY(hipSetDevice(h->device));
    f();
    return CHEFSI_OK;
  } catch (const Error& e) {
    return fail(h, e);
  } catch (const std::bad_alloc&) {
    return fail(h, Error{CHEFSI_ERR_OOM, "host allocation failed"});
  } catch (...) {
    return fail(h, Error{CHEFSI_ERR_HIP, "unexpected exception"});
  }
}

template <typename T>
T* upload(chefsi_handle* h, const T* src, size_t n) {
  T* d = nullptr;
  if (n == 0) return nullptr;
  h->device_bytes += n * sizeof(T);
  if (hipMalloc(&d, n * sizeof(T)) != hipSuccess) throw Error{CHEFSI_ERR_OOM, "device allocation failed"};
  hipError_t e = hipMemcpy(d, src, n * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    throw Error{CHEFSI_ERR_HIP, std::string("upload: ") + hipGetErrorString(e)};
  }
  return d;
}

// Stencil-pass projector records for tiling hp (points in one to four projector entries,
// grouped by (y tile, z plane); at most ty * nx per group <= PY * threads), replacing the
// handle's current ones.  The LDS budget (the alpha row and the partial-sum buffers
// beside the tile) is checked for the longest z chunk (zc = nz), which the planner picks
// for wide blocks; with no records (band route) the pass carries neither.
static bool hx_records_fit(const chefsi_handle* h, const HxPlan& hp) {
  HxPlan worst = hp;
  worst.zc = h->n[2];
  const int nx = h->n[0];
  const size_t lds_need = std::max(hx_lds_bytes(worst, nx, h->radius, h->precision == CHEFSI_FP64 ? 8 : 4,
                                                h->np_tot, 8),
                                   hx_lds_bytes(worst, nx, h->radius, 4, h->np_tot, 8));
  return lds_need <= kHxMaxLds;
}

void build_hx_records(chefsi_handle* h, const HxPlan& hp) {
  const int nx = h->n[0], ny = h->n[1], nz = h->n[2];
  const int64_t nd = h->nd;
  check(h->rec_max == 0 || hx_records_fit(h, hp),
        "too many projectors for the stencil pass (alpha row does not fit in LDS)");
  const int64_t nkeys = (int64_t)hp.nty * nz;
  auto key_of = [&](int64_t i) {
    const int y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    return (int64_t)(y / hp.ty) * nz + z;
  };
  const std::vector<int>& cnt = h->pt_cnt;
  std::vector<int> rptr(nkeys + 1, 0);
  for (int64_t i = 0; i < nd; ++i) {
    const int n = cnt[i + 1] - cnt[i];
    if (n >= 1 && n <= h->rec_max) rptr[key_of(i) + 1] += 1;
  }
  for (int64_t k = 0; k < nkeys; ++k) rptr[k + 1] += rptr[k];
  const int nrec = rptr[nkeys];
  std::vector<HxRec<double>> r64(std::max(nrec, 1));
  std::vector<HxRec<float>> r32(std::max(nrec, 1));
  std::memset(r64.data(), 0, r64.size() * sizeof(HxRec<double>));
  std::memset(r32.data(), 0, r32.size() * sizeof(HxRec<float>));
  std::vector<int> rfill(rptr.begin(), rptr.end() - 1);
  for (int64_t i = 0; i < nd; ++i) {
    const int b = cnt[i], n = cnt[i + 1] - b;
    if (n < 1 || n > h->rec_max) continue;
    const int r = rfill[key_of(i)]++;
    const int x = (int)(i % nx), y = (int)((i / nx) % ny);
    int col[4] = {0, 0, 0, 0};
    for (int k = 0; k < n; ++k) {
      col[k] = h->pt_col[b + k];
      r64[r].val[k] = h->pt_val[b + k];
      r32[r].val[k] = (float)h->pt_val[b + k];
    }
    r64[r].lidx = r32[r].lidx = (y % hp.ty) * nx + x;
    r64[r].c01 = r32[r].c01 = col[0] | (col[1] << 16);
    r64[r].c23 = r32[r].c23 = col[2] | (col[3] << 16);
  }
  int* nptr = nullptr;
  HxRec<double>* n64 = nullptr;
  HxRec<float>* n32 = nullptr;
  try {
    if (nrec > 0) {
      nptr = upload(h, rptr.data(), rptr.size());
      n64 = upload(h, r64.data(), r64.size());
      n32 = upload(h, r32.data(), r32.size());
    }
  } catch (...) {
    for (void* q : {(void*)nptr, (void*)n64, (void*)n32})
      if (q) (void)hipFree(q);
    throw;
  }
  for (void* q : {(void*)h->hx_rec_ptr, (void*)h->hx_rec64, (void*)h->hx_rec32})
    if (q) (void)hipFree(q);
  h->device_bytes -= h->hx_rec_bytes;
  h->hx_rec_bytes = nrec > 0 ? rptr.size() * sizeof(int) + r64.size() * sizeof(HxRec<double>) +
                                   r32.size() * sizeof(HxRec<float>)
                             : 0;
  h->hx_rec_ptr = nptr;
  h->hx_rec64 = n64;
  h->hx_rec32 = n32;
  h->n_hxrec = nrec;
  h->hx_plan = hp;
}

void free_band_tables(chefsi_handle* h) {
  void* ptrs[] = {h->nb_reg_pt,   h->nb_pt_idx,     h->nb_pt_ent,     h->nb_ent_ls,   h->nb_ent_chi64,
                  h->nb_ent_chi32, h->nb_reg_slot,  h->nb_slot_ent,   h->nb_gent_loc, h->nb_gent_chi64,
                  h->nb_gent_chi32, h->nb_q_slot_ptr, h->nb_q_slot,   h->nb_partial, h->nb_slot_q};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  h->nb_reg_pt = h->nb_pt_idx = h->nb_pt_ent = h->nb_ent_ls = h->nb_slot_q = nullptr;
  h->nb_reg_slot = h->nb_slot_ent = h->nb_gent_loc = h->nb_q_slot_ptr = h->nb_q_slot = nullptr;
  h->nb_ent_chi64 = h->nb_gent_chi64 = nullptr;
  h->nb_ent_chi32 = h->nb_gent_chi32 = nullptr;
  h->nb_partial = nullptr;
  h->device_bytes -= h->nb_bytes;
  h->nb_bytes = 0;
  h->nb_reg = h->nb_pts = h->nb_slots = 0;
}

// Band-pass regions from a point-major projector table (cnt: nd + 1 entry offsets, col: the
// projector column of every entry): regions of consecutive touched points (grid index
// order), each closed before it would exceed kBandMaxPts points, kBandMaxSlots projectors or
// max_ent entries; each region lists its points with their entries, and its projector slots
// (projector order) with their entries (point order); each projector lists its slots (region
// order) for the reduction.  ent_src / gent_src name the table entry behind every scatter /
// gather entry, so the caller attaches values of its own type.
struct BandRegions {
  std::vector<int> reg_pt{0}, pt_idx, pt_ent{0}, ent_ls, reg_slot{0}, slot_q, slot_ent{0}, gent_loc, q_slot_ptr{0},
      q_slot, ent_src, gent_src;
};

BandRegions band_regions(int64_t nd, const int* cnt, const int* col, int np_tot, int max_ent) {
  BandRegions R;
  std::vector<std::vector<int>> q_slots(np_tot);
  std::vector<int64_t> open;              // points of the open region
  std::vector<int> stamp(np_tot, -1);     // region that last counted each projector
  int nreg = 0, open_ent = 0, open_q = 0;
  auto close_region = [&]() {
    const int first = (int)R.pt_idx.size();
    std::map<int, std::vector<std::pair<int, int>>> slots;  // projector -> (local point, table entry)
    const size_t e_first = R.ent_src.size();
    for (int64_t i : open) {
      const int loc = (int)R.pt_idx.size() - first;
      R.pt_idx.push_back((int)i);
      for (int e = cnt[i]; e < cnt[i + 1]; ++e) {
        R.ent_src.push_back(e);
        slots[col[e]].emplace_back(loc, e);
      }
      R.pt_ent.push_back((int)R.ent_src.size());
    }
    R.reg_pt.push_back((int)R.pt_idx.size());
    std::map<int, int> local;  // region slot of every entry (slots in projector order)
    for (auto& kv : slots) local.emplace(kv.first, (int)local.size());
    for (size_t e = e_first; e < R.ent_src.size(); ++e) R.ent_ls.push_back(local.at(col[R.ent_src[e]]));
    for (auto& kv : slots) {
      q_slots[kv.first].push_back((int)R.slot_q.size());
      R.slot_q.push_back(kv.first);
      for (auto& pe : kv.second) {
        R.gent_loc.push_back(pe.first);
        R.gent_src.push_back(pe.second);
      }
      R.slot_ent.push_back((int)R.gent_loc.size());
    }
    R.reg_slot.push_back((int)R.slot_q.size());
    open.clear();
    open_ent = open_q = 0;
    ++nreg;
  };
  for (int64_t i = 0; i < nd; ++i) {
    const int n = cnt[i + 1] - cnt[i];
    if (n == 0) continue;
    check(n <= kBandMaxSlots && n <= max_ent, "a grid point lies in too many projector supports for the band pass");
    int fresh = 0;
    for (int e = cnt[i]; e < cnt[i + 1]; ++e) fresh += stamp[col[e]] != nreg;
    if (!open.empty() &&
        ((int)open.size() + 1 > kBandMaxPts || open_ent + n > max_ent || open_q + fresh > kBandMaxSlots)) {
      close_region();
      fresh = n;  // every projector of the point is new to the next region
    }
    for (int e = cnt[i]; e < cnt[i + 1]; ++e) stamp[col[e]] = nreg;
    open.push_back(i);
    open_ent += n;
    open_q += fresh;
  }
  if (!open.empty()) close_region();
  for (int q = 0; q < np_tot; ++q) {
    for (int sl : q_slots[q]) R.q_slot.push_back(sl);
    R.q_slot_ptr.push_back((int)R.q_slot.size());
  }
  return R;
}

// Band-pass tables of a real handle (FP64 and FP32 copies of the projector values).
void build_band_tables(chefsi_handle* h) {
  free_band_tables(h);
  BandRegions R = band_regions(h->nd, h->pt_cnt.data(), h->pt_col.data(), h->np_tot, kBandMaxEnt);
  std::vector<double> ent_chi(R.ent_src.size()), gent_chi(R.gent_src.size());
  for (size_t e = 0; e < ent_chi.size(); ++e) ent_chi[e] = h->pt_val[R.ent_src[e]];
  for (size_t e = 0; e < gent_chi.size(); ++e) gent_chi[e] = h->pt_val[R.gent_src[e]];
  const std::vector<int>& reg_pt = R.reg_pt;
  const std::vector<int>& pt_idx = R.pt_idx;
  const std::vector<int>& pt_ent = R.pt_ent;
  const std::vector<int>& ent_ls = R.ent_ls;
  const std::vector<int>& slot_q = R.slot_q;
  const std::vector<int>& reg_slot = R.reg_slot;
  const std::vector<int>& slot_ent = R.slot_ent;
  const std::vector<int>& gent_loc = R.gent_loc;
  const std::vector<int>& q_slot_ptr = R.q_slot_ptr;
  const std::vector<int>& q_slot = R.q_slot;
  const size_t before = h->device_bytes;
  try {
    h->nb_reg_pt = upload(h, reg_pt.data(), reg_pt.size());
    h->nb_pt_idx = upload(h, pt_idx.data(), pt_idx.size());
    h->nb_pt_ent = upload(h, pt_ent.data(), pt_ent.size());
    h->nb_ent_ls = upload(h, ent_ls.data(), ent_ls.size());
    h->nb_slot_q = upload(h, slot_q.data(), slot_q.size());
    h->nb_ent_chi64 = upload(h, ent_chi.data(), ent_chi.size());
    std::vector<float> f(ent_chi.begin(), ent_chi.end());
    h->nb_ent_chi32 = upload(h, f.data(), f.size());
    h->nb_reg_slot = upload(h, reg_slot.data(), reg_slot.size());
    h->nb_slot_ent = upload(h, slot_ent.data(), slot_ent.size());
    h->nb_gent_loc = upload(h, gent_loc.data(), gent_loc.size());
    h->nb_gent_chi64 = upload(h, gent_chi.data(), gent_chi.size());
    std::vector<float> g(gent_chi.begin(), gent_chi.end());
    h->nb_gent_chi32 = upload(h, g.data(), g.size());
    h->nb_q_slot_ptr = upload(h, q_slot_ptr.data(), q_slot_ptr.size());
    h->nb_q_slot = upload(h, q_slot.data(), q_slot.size());
    const size_t pbytes = std::max<size_t>(1, slot_q.size()) * (size_t)h->max_ns * 8;
    if (hipMalloc(&h->nb_partial, pbytes) != hipSuccess) {
      h->nb_partial = nullptr;
      throw Error{CHEFSI_ERR_OOM, "device allocation failed (band-pass partial sums)"};
    }
    h->device_bytes += pbytes;
  } catch (...) {
    h->nb_bytes = h->device_bytes - before;
    free_band_tables(h);
    throw;
  }
  h->nb_bytes = h->device_bytes - before;
  h->nb_reg = (int)reg_pt.size() - 1;
  h->nb_pts = (int)pt_idx.size();
  h->nb_slots = (int)slot_q.size();
}

// Scatter-pass records for the points in more than rec_max projector entries (all touched
// points when rec_max is 0): one record {point, first entry, entry count, 0} each, entries
// in atom order padded with zeros to a multiple of 4; replaces the handle's current ones.
void build_scatter_records(chefsi_handle* h) {
  std::vector<int4> recs;
  const bool band = h->rec_max == 0;  // the band pass takes every term: no scatter records
  std::vector<int> ecol;
  std::vector<double> evals;
  for (int64_t i = 0; i < h->nd; ++i) {
    const int b = h->pt_cnt[i], n = h->pt_cnt[i + 1] - b;
    if (band || n <= h->rec_max) continue;
    recs.push_back(make_int4((int)i, (int)ecol.size(), n, 0));
    for (int k = b; k < b + n; ++k) {
      ecol.push_back(h->pt_col[k]);
      evals.push_back(h->pt_val[k]);
    }
    while (ecol.size() % 4) {
      ecol.push_back(0);
      evals.push_back(0.0);
    }
  }
  check(ecol.size() < ((size_t)1 << 31), "too many projector entries");
  int4* rec = nullptr;
  int* col = nullptr;
  double* v64 = nullptr;
  float* v32 = nullptr;
  try {
    if (!recs.empty()) {
      rec = upload(h, recs.data(), recs.size());
      col = upload(h, ecol.data(), ecol.size());
      v64 = upload(h, evals.data(), evals.size());
      std::vector<float> ev32(evals.begin(), evals.end());
      v32 = upload(h, ev32.data(), ev32.size());
    }
  } catch (...) {
    for (void* q : {(void*)rec, (void*)col, (void*)v64, (void*)v32})
      if (q) (void)hipFree(q);
    throw;
  }
  for (void* q : {(void*)h->rec, (void*)h->ent_col, (void*)h->ent_val64, (void*)h->ent_val32})
    if (q) (void)hipFree(q);
  h->device_bytes -= h->scatter_bytes;
  h->scatter_bytes = recs.empty() ? 0
                                  : recs.size() * sizeof(int4) + ecol.size() * (sizeof(int) + sizeof(double) +
                                                                                sizeof(float));
  h->rec = rec;
  h->ent_col = col;
  h->ent_val64 = v64;
  h->ent_val32 = v32;
  h->n_pts = (int)recs.size();
}

void release(chefsi_handle* h) {
  free_band_tables(h);
  void* ptrs[] = {h->veff64, h->veff32, h->supp_off, h->supp_idx, h->chi_off,  h->nproj,    h->poff,
                  h->chi64,  h->chi32,  h->gdv64,    h->gdv32,    h->rec,      h->ent_col,  h->hx_rec_ptr,
                  h->hx_rec64, h->hx_rec32,
                  h->ent_val64,
                  h->ent_val32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& p : h->ev_pending) {
    (void)hipEventDestroy(p.b);
    (void)hipEventDestroy(p.e);
  }
  for (auto ev : h->ev_pool) (void)hipEventDestroy(ev);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->blas) rocblas_destroy_handle(h->blas);
}

}  // namespace

extern "C" {

int chefsi_version(void) { return 100; }

const char* chefsi_strerror(int status) {
  switch (status) {
    case CHEFSI_OK: return "ok";
    case CHEFSI_ERR_INVALID_ARG: return "invalid argument";
    case CHEFSI_ERR_HIP: return "HIP runtime error";
    case CHEFSI_ERR_WORKSPACE: return "workspace too small";
    case CHEFSI_ERR_NOT_POSDEF: return "overlap matrix not positive definite";
    case CHEFSI_ERR_EIG: return "dense eigensolver did not converge";
    case CHEFSI_ERR_NONFINITE: return "non-finite Ritz value";
    case CHEFSI_ERR_SOLVER: return "rocBLAS/rocSOLVER error";
    case CHEFSI_ERR_OOM: return "out of memory";
    default: return "unknown status";
  }
}

const char* chefsi_last_error(const chefsi_handle_t* h) { return h ? h->last_error.c_str() : ""; }

int chefsi_last_info(const chefsi_handle_t* h) { return h ? h->last_info : 0; }

int chefsi_update_veff(chefsi_handle_t* h, const double* veff_host, void* stream) {
  return guarded(h, [&] {
    check(veff_host != nullptr, "veff_host is NULL");
    for (int64_t i = 0; i < h->nd; ++i) check(std::isfinite(veff_host[i]), "Veff must be finite");
    hipStream_t s = (hipStream_t)stream;
    h->veff_h.assign(veff_host, veff_host + h->nd);
    const std::vector<float> v32(h->veff_h.begin(), h->veff_h.end());
    HIP_TRY(hipMemcpyAsync(h->veff64, h->veff_h.data(), (size_t)h->nd * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->veff32, v32.data(), (size_t)h->nd * sizeof(float), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // v32 and the caller's array may go away after return
  });
}

int chefsi_create(const chefsi_grid_t* grid, const double* veff_host, const chefsi_nonlocal_t* nl,
                  int32_t precision, int32_t max_ns, chefsi_handle_t** out) {
  if (out == nullptr) return CHEFSI_ERR_INVALID_ARG;
  *out = nullptr;
  if (grid == nullptr || veff_host == nullptr) return CHEFSI_ERR_INVALID_ARG;
  chefsi_handle* h = nullptr;
  try {
    h = new chefsi_handle();
  } catch (...) {
    return CHEFSI_ERR_OOM;
  }
  try {
    check(precision == CHEFSI_FP64 || precision == CHEFSI_MIXED, "precision must be CHEFSI_FP64 or CHEFSI_MIXED");
    check(grid->fd_order >= 2 && grid->fd_order <= 12 && grid->fd_order % 2 == 0, "fd_order must be even, 2..12");
    h->precision = precision;
    h->order = grid->fd_order;
    h->radius = grid->fd_order / 2;
    int64_t nd = 1;
    for (int d = 0; d < 3; ++d) {
      check(grid->n[d] >= 1, "grid sizes must be >= 1");
      check(grid->bc[d] == 0 || grid->bc[d] == 1, "bc must be 0 (periodic) or 1 (Dirichlet)");
      check(std::isfinite(grid->h[d]) && grid->h[d] > 0.0, "grid spacing must be positive");
      if (grid->bc[d] == 0) check(grid->n[d] >= h->radius, "periodic direction needs n >= fd_order/2");
      h->n[d] = grid->n[d];
      h->h[d] = grid->h[d];
      h->bc[d] = grid->bc[d];
      nd *= grid->n[d];
    }
    check(nd < (int64_t)1 << 31, "Nd must be below 2^31");
    // the stencil pass addresses one orbital, Veff and the projector records (48 bytes per
    // point at most) through buffer resources of fewer than 2^31 bytes
    check(nd * 48 < (int64_t)1 << 31, "grids above 44 million points are not supported by the stencil pass");
    check(grid->n[0] <= kHxMaxThreads, "nx above 512 is not supported by the stencil tiling");
    check(max_ns >= 1 && (int64_t)max_ns <= nd, "max_ns must satisfy 1 <= max_ns <= Nd");
    for (int eb : {4, 8})
      check(plan_hx(grid->n[0], grid->n[1], grid->n[2], 1, grid->fd_order / 2, eb, 0, 0).ok,
            "grid too wide in x for the stencil tiling (the halo rows of a tile need at most four values per thread)");
    h->nd = nd;
    h->max_ns = max_ns;
    h->dv = grid->h[0] * grid->h[1] * grid->h[2];
    h->w = fd_weights(h->order);
    h->veff_h.assign(veff_host, veff_host + nd);
    for (double v : h->veff_h) check(std::isfinite(v), "Veff must be finite");

    // projectors
    if (nl != nullptr && nl->n_atoms > 0) {
      check(nl->supp_ptr && nl->supp_idx && nl->nproj && nl->chi && nl->gamma, "null projector array");
      const int na = nl->n_atoms;
      h->n_atoms = na;
      h->supp_ptr_h.assign(nl->supp_ptr, nl->supp_ptr + na + 1);
      check(h->supp_ptr_h[0] == 0, "supp_ptr[0] must be 0");
      for (int J = 0; J < na; ++J) check(h->supp_ptr_h[J + 1] >= h->supp_ptr_h[J], "supp_ptr must be non-decreasing");
      const int64_t nsupp = h->supp_ptr_h[na];
      check(nsupp < (int64_t)1 << 31, "too many support points");
      h->supp_idx_h.assign(nl->supp_idx, nl->supp_idx + nsupp);
      h->nproj_h.assign(nl->nproj, nl->nproj + na);
      int64_t nchi = 0, npt = 0;
      for (int J = 0; J < na; ++J) {
        check(h->nproj_h[J] >= 1, "nproj must be >= 1");
        const int64_t nj = h->supp_ptr_h[J + 1] - h->supp_ptr_h[J];
        for (int64_t s = 0; s < nj; ++s) {
          const int64_t i = h->supp_idx_h[h->supp_ptr_h[J] + s];
          check(i >= 0 && i < nd, "support index outside the grid");
          if (s > 0) check(i > h->supp_idx_h[h->supp_ptr_h[J] + s - 1], "support indices must increase");
        }
        nchi += nj * h->nproj_h[J];
        npt += h->nproj_h[J];
      }
      check(npt < (int64_t)1 << 30 && nchi < ((int64_t)1 << 40), "too many projectors");
      h->np_tot = (int)npt;
      h->chi_h.assign(nl->chi, nl->chi + nchi);
      h->gamma_h.assign(nl->gamma, nl->gamma + npt);
      for (double v : h->chi_h) check(std::isfinite(v), "chi must be finite");
      for (double v : h->gamma_h) check(std::isfinite(v), "gamma must be finite");
    }

    HIP_TRY(hipGetDevice(&h->device));
    (void)scratch_address(h->device);  // the static scratch's device address, once per device
    BLAS_TRY(rocblas_create_handle(&h->blas));
    // the dense stage must give the same bits whatever else runs on the device (results of
    // a request alone and among others are compared bit for bit): no atomics in rocBLAS
    BLAS_TRY(rocblas_set_atomics_mode(h->blas, rocblas_atomics_not_allowed));
    h->hx_plan = plan_hx(h->n[0], h->n[1], h->n[2], 1, h->radius, precision == CHEFSI_FP64 ? 8 : 4, 0, 0);
    check(h->hx_plan.ok, "no stencil tiling fits this grid");

    if (hipHostMalloc((void**)&h->pinned, (size_t)max_ns * sizeof(double) + 64, hipHostMallocDefault) != hipSuccess) {
      h->pinned = nullptr;
      throw Error{CHEFSI_ERR_OOM, "pinned host allocation failed"};
    }
    h->veff64 = upload(h, h->veff_h.data(), nd);
    std::vector<float> v32(h->veff_h.begin(), h->veff_h.end());
    h->veff32 = upload(h, v32.data(), nd);

    if (h->np_tot > 0) {
      const int na = h->n_atoms;
      std::vector<int> soff(na + 1), poff(na);
      std::vector<int64_t> coff(na);
      int64_t c = 0;
      int p = 0;
      for (int J = 0; J < na; ++J) {
        soff[J] = (int)h->supp_ptr_h[J];
        coff[J] = c;
        poff[J] = p;
        c += (h->supp_ptr_h[J + 1] - h->supp_ptr_h[J]) * h->nproj_h[J];
        p += h->nproj_h[J];
      }
      soff[na] = (int)h->supp_ptr_h[na];
      std::vector<double> gdv(h->np_tot);
      for (int q = 0; q < h->np_tot; ++q) gdv[q] = h->gamma_h[q] * h->dv;
      // point-major table: point i lists (projector column, chi value), atoms in order
      std::vector<int> cnt(nd + 1, 0);
      for (int J = 0; J < na; ++J)
        for (int64_t s = h->supp_ptr_h[J]; s < h->supp_ptr_h[J + 1]; ++s) cnt[h->supp_idx_h[s] + 1] += h->nproj_h[J];
      for (int64_t i = 0; i < nd; ++i) cnt[i + 1] += cnt[i];
      const int64_t nent = cnt[nd];
      check(nent < (int64_t)1 << 31, "too many projector entries");
      std::vector<int> fill(cnt.begin(), cnt.end() - 1), eproj(nent);
      std::vector<double> eval(nent);
      for (int J = 0; J < na; ++J) {
        const int64_t nj = h->supp_ptr_h[J + 1] - h->supp_ptr_h[J];
        for (int64_t s = 0; s < nj; ++s) {
          const int i = h->supp_idx_h[h->supp_ptr_h[J] + s];
          for (int a = 0; a < h->nproj_h[J]; ++a) {
            const int pos = fill[i]++;
            eproj[pos] = poff[J] + a;
            eval[pos] = h->chi_h[coff[J] + a * nj + s];
          }
        }
      }
      h->pt_cnt = std::move(cnt);
      h->pt_col = std::move(eproj);
      h->pt_val = std::move(eval);
      check(h->np_tot < 65536, "more than 65535 projectors");
      // the record route keeps the block's projector row and partial sums in LDS beside the
      // tile; a handle whose projectors overflow that budget for the default tile starts on
      // the band pass
      if (!hx_records_fit(h, h->hx_plan)) {
        try {
          build_band_tables(h);
        } catch (const Error& e) {
          throw Error{e.status, "too many projectors for the stencil pass (alpha row does not fit in LDS), and " + e.msg};
        }
        h->rec_max = 0;
      }
      build_hx_records(h, h->hx_plan);
      build_scatter_records(h);
      h->supp_off = upload(h, soff.data(), soff.size());
      h->supp_idx = upload(h, h->supp_idx_h.data(), h->supp_idx_h.size());
      h->chi_off = upload(h, coff.data(), coff.size());
      h->nproj = upload(h, h->nproj_h.data(), h->nproj_h.size());
      h->poff = upload(h, poff.data(), poff.size());
      h->chi64 = upload(h, h->chi_h.data(), h->chi_h.size());
      std::vector<float> chi32(h->chi_h.begin(), h->chi_h.end());
      h->chi32 = upload(h, chi32.data(), chi32.size());
      h->gdv64 = upload(h, gdv.data(), gdv.size());
      std::vector<float> gdv32(gdv.begin(), gdv.end());
      h->gdv32 = upload(h, gdv32.data(), gdv32.size());
    }
    *out = h;
    return CHEFSI_OK;
  } catch (const Error& e) {
    release(h);
    delete h;
    return e.status;
  } catch (const std::bad_alloc&) {
    release(h);
    delete h;
    return CHEFSI_ERR_OOM;
  } catch (...) {
    release(h);
    delete h;
    return CHEFSI_ERR_HIP;
  }
}

void chefsi_destroy(chefsi_handle_t* h) {
  if (!h) return;
  release(h);
  delete h;
}

int chefsi_workspace_bytes(const chefsi_handle_t* hc, int32_t ns, size_t* bytes) {
  chefsi_handle* h = const_cast<chefsi_handle*>(hc);
  return guarded(h, [&] {
    check(bytes != nullptr, "bytes is NULL");
    check_ns(h, ns);
    *bytes = layout(h, ns).total;
  });
}

int chefsi_spectral_bounds(const chefsi_handle_t* hc, double* lam_lo, double* lam_cut, double* lam_hi) {
  chefsi_handle* h = const_cast<chefsi_handle*>(hc);
  return guarded(h, [&] {
    double s = std::fabs(h->w[0]);
    for (int p = 1; p <= h->radius; ++p) s += 2.0 * std::fabs(h->w[p]);
    double kin = 0.0;
    for (int d = 0; d < 3; ++d) kin += 0.5 * s / (h->h[d] * h->h[d]);
    double vmax = -INFINITY, vmin = INFINITY;
    for (double v : h->veff_h) {
      vmax = std::max(vmax, v);
      vmin = std::min(vmin, v);
    }
    std::vector<double> row(h->nd, 0.0);
    bool negative = false;
    int64_t coff = 0;
    int q = 0;
    for (int J = 0; J < h->n_atoms; ++J) {
      const int64_t s0 = h->supp_ptr_h[J], nj = h->supp_ptr_h[J + 1] - s0;
      for (int a = 0; a < h->nproj_h[J]; ++a, ++q) {
        const double* c = h->chi_h.data() + coff + a * nj;
        double l1 = 0.0;
        for (int64_t t = 0; t < nj; ++t) l1 += std::fabs(c[t]);
        const double g = std::fabs(h->gamma_h[q]);
        if (h->gamma_h[q] < 0) negative = true;
        for (int64_t t = 0; t < nj; ++t) row[h->supp_idx_h[s0 + t]] += g * std::fabs(c[t]) * l1 * h->dv;
      }
      coff += nj * h->nproj_h[J];
    }
    double nlb = 0.0;
    for (double v : row) nlb = std::max(nlb, v);
    const double hi = kin + vmax + nlb;
    const double lo = vmin - (negative ? nlb : 0.0);
    if (lam_hi) *lam_hi = hi;
    if (lam_lo) *lam_lo = lo;
    if (lam_cut) *lam_cut = lo + 0.1 * (hi - lo);
  });
}

int chefsi_static_scratch_bytes(const chefsi_handle_t* h, int32_t ns, size_t* bytes) {
  if (h == nullptr || bytes == nullptr || ns < 1) return CHEFSI_ERR_INVALID_ARG;
  *bytes = (size_t)h->np_tot * (size_t)ns * (h->precision == CHEFSI_FP64 ? sizeof(double) : sizeof(float));
  return CHEFSI_OK;
}

int chefsi_apply_h_static(chefsi_handle_t* h, const void* X, void* Y, int32_t ns, void* stream) {
  return guarded(h, [&] {
    check(X != nullptr && Y != nullptr && X != Y, "X and Y must be distinct device blocks");
    check_ns(h, ns);
    size_t need = 0;
    (void)chefsi_static_scratch_bytes(h, ns, &need);
    if (need > (size_t)CHEFSI_STATIC_SCRATCH_BYTES)
      throw Error{CHEFSI_ERR_WORKSPACE, "np_tot x ns projector coefficients (" + std::to_string(need) +
                                            " bytes) exceed the static scratch of " +
                                            std::to_string((size_t)CHEFSI_STATIC_SCRATCH_BYTES) +
                                            " bytes: call on fewer orbitals at a time"};
    void* alpha = scratch_address(h->device);  // looked up at create; a table read here
    hipStream_t s = (hipStream_t)stream;
    // no event records either (profiling may create events): the call only enqueues kernels
    const bool prof = h->prof_on;
    h->prof_on = false;
    struct Restore {
      chefsi_handle* h;
      bool v;
      ~Restore() { h->prof_on = v; }
    } restore{h, prof};
    if (h->precision == CHEFSI_FP64)
      apply_fused<double, double, double>(h, (const double*)X, nullptr, (double*)Y, ns, 1.0, 0.0, 0.0,
                                          (double*)alpha, s);
    else
      apply_fused<float, float, float>(h, (const float*)X, nullptr, (float*)Y, ns, 1.0, 0.0, 0.0, (float*)alpha,
                                       s);
  });
}

int chefsi_apply_h(chefsi_handle_t* h, const void* X, void* Y, int32_t ns, void* ws, size_t ws_bytes, void* stream) {
  return guarded(h, [&] {
    check(X != nullptr && Y != nullptr && X != Y, "X and Y must be distinct device blocks");
    check_ns(h, ns);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64)
      apply_fused<double, double, double>(h, (const double*)X, nullptr, (double*)Y, ns, 1.0, 0.0, 0.0,
                                          at<double>(ws, L.alpha), s);
    else
      apply_fused<float, float, float>(h, (const float*)X, nullptr, (float*)Y, ns, 1.0, 0.0, 0.0,
                                       at<float>(ws, L.alpha), s);
  });
}

int chefsi_filter(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree, double lam_lo, double lam_cut,
                  double lam_hi, void* ws, size_t ws_bytes, void* stream) {
  return guarded(h, [&] {
    check(X != nullptr, "X is NULL");
    check(degree >= 1, "degree must be >= 1");
    check_ns(h, ns);
    check_bounds(lam_lo, lam_cut, lam_hi);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64) {
      double* A = (double*)X;
      double* r = run_filter<double>(h, A, at<double>(ws, L.bufB), ns, degree, lam_lo, lam_cut, lam_hi,
                                     at<double>(ws, L.alpha), s);
      if (r != A) copy_block<double>(h, A, r, ns, s);
    } else {
      float* A = (float*)X;
      float* r = run_filter<float>(h, A, at<float>(ws, L.bufB), ns, degree, lam_lo, lam_cut, lam_hi,
                                   at<float>(ws, L.alpha), s);
      if (r != A) copy_block<float>(h, A, r, ns, s);
    }
  });
}

int chefsi_project(chefsi_handle_t* h, const void* X, int32_t ns, double* Hs, double* Ms, void* ws,
                   size_t ws_bytes, void* stream) {
  return guarded(h, [&] {
    check(X != nullptr && Hs != nullptr && Ms != nullptr, "null pointer");
    check_ns(h, ns);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64) {
      double* Y = at<double>(ws, L.bufB);
      apply_fused<double, double, double>(h, (const double*)X, nullptr, Y, ns, 1.0, 0.0, 0.0,
                                          at<double>(ws, L.alpha), s);
      gram_pair<double, double>(h, (const double*)X, Y, ns, L, ws, Hs, Ms, s, Gemm::F64);
    } else {
      float* Y = at<float>(ws, L.bufB);
      apply_fused<float, float, float>(h, (const float*)X, nullptr, Y, ns, 1.0, 0.0, 0.0, at<float>(ws, L.alpha),
                                       s);
      gram_pair<float, float>(h, (const float*)X, Y, ns, L, ws, Hs, Ms, s, Gemm::BF16X3);
    }
  });
}

int chefsi_eigh(chefsi_handle_t* h, double* Hs, double* Ms, double* D, int32_t ns, void* ws, size_t ws_bytes,
                void* stream) {
  return guarded(h, [&] {
    check(Hs != nullptr && Ms != nullptr && D != nullptr, "null pointer");
    check_ns(h, ns);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    dense_eig(h, Hs, Ms, D, ns, L, ws, s);
    check_info(h, ws, L, ns, s);
  });
}

int chefsi_rotate(chefsi_handle_t* h, void* X, const double* Z, int32_t ns, void* ws, size_t ws_bytes,
                  void* stream) {
  return guarded(h, [&] {
    check(X != nullptr && Z != nullptr, "null pointer");
    check_ns(h, ns);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64) {
      double* B = at<double>(ws, L.bufB);
      rotate_into<double>(h, (const double*)X, Z, B, ns, s, Gemm::F64, ws, L);
      copy_block<double>(h, (double*)X, B, ns, s);
    } else {
      float* B = at<float>(ws, L.bufB);
      rotate_into<float>(h, (const float*)X, Z, B, ns, s, Gemm::BF16X3, ws, L);
      copy_block<float>(h, (float*)X, B, ns, s);
    }
  });
}

int chefsi_step(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree, double lam_lo, double lam_cut,
                double lam_hi, void* ws, size_t ws_bytes, void* stream, double* ritz_host) {
  return guarded(h, [&] {
    check(X != nullptr, "X is NULL");
    check(degree >= 1, "degree must be >= 1");
    check_ns(h, ns);
    check_bounds(lam_lo, lam_cut, lam_hi);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64)
      step_impl<double>(h, (double*)X, ns, degree, lam_lo, lam_cut, lam_hi, ws, L, s, ritz_host);
    else
      step_impl<float>(h, (float*)X, ns, degree, lam_lo, lam_cut, lam_hi, ws, L, s, ritz_host);
  });
}

int chefsi_solve(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree, int32_t n_iter, double lam_lo,
                 double lam_cut, double lam_hi, void* ws, size_t ws_bytes, void* stream, double* ritz_host,
                 double* lam_lo_out, double* lam_cut_out) {
  return guarded(h, [&] {
    check(X != nullptr, "X is NULL");
    check(degree >= 1 && n_iter >= 1, "degree and n_iter must be >= 1");
    check_ns(h, ns);
    check_bounds(lam_lo, lam_cut, lam_hi);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> d(ns);
    double lo = lam_lo, cut = lam_cut;
    for (int it = 0; it < n_iter; ++it) {
      check_bounds(lo, cut, lam_hi);
      if (h->precision == CHEFSI_FP64)
        step_impl<double>(h, (double*)X, ns, degree, lo, cut, lam_hi, ws, L, s, d.data());
      else
        step_impl<float>(h, (float*)X, ns, degree, lo, cut, lam_hi, ws, L, s, d.data());
      lo = d[0];
      cut = d[ns - 1];
    }
    if (ritz_host) std::memcpy(ritz_host, d.data(), (size_t)ns * 8);
    if (lam_lo_out) *lam_lo_out = lo;
    if (lam_cut_out) *lam_cut_out = cut;
  });
}

int chefsi_refine_fp64(chefsi_handle_t* h, void* X, int32_t ns, int32_t degree, double lam_lo, double lam_cut,
                       double lam_hi, void* ws, size_t ws_bytes, void* stream, double* ritz_host) {
  return guarded(h, [&] {
    check(X != nullptr, "X is NULL");
    check(degree >= 0, "degree must be >= 0");
    check_ns(h, ns);
    if (degree > 0) check_bounds(lam_lo, lam_cut, lam_hi);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64)
      refine_impl<double>(h, (double*)X, ns, degree, lam_lo, lam_cut, lam_hi, ws, L, s, ritz_host);
    else
      refine_impl<float>(h, (float*)X, ns, degree, lam_lo, lam_cut, lam_hi, ws, L, s, ritz_host);
  });
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Lanczos estimate of lam_Nd (Alg. 1: the largest eigenvalue of H).
// Workspace: v_{j-1}, v_j (storage type), w (FP64), the projector coefficients of one
// vector (FP64), the block sums and two result words.
// ---------------------------------------------------------------------------
struct LzLayout {
  size_t v0 = 0, v1 = 0, w = 0, alpha = 0, partial = 0, out = 0, total = 0;
};

LzLayout lanczos_layout(const chefsi_handle* h) {
  LzLayout L;
  const size_t vb = (size_t)h->nd * elem_bytes(h);
  size_t off = 0;
  L.v0 = off;
  off += align256(vb);
  L.v1 = off;
  off += align256(vb);
  L.w = off;
  off += align256((size_t)h->nd * 8);
  L.alpha = off;
  off += align256((size_t)std::max(1, h->np_tot) * 8);
  L.partial = off;
  off += align256((size_t)kVecBlocks * 8);
  L.out = off;
  off += 256;
  L.total = off;
  return L;
}

// Largest eigenvalue theta of the symmetric tridiagonal T (diagonal a[0..k), off-diagonal
// b[0..k-1)) by Sturm-count bisection to full precision, and the last component of its
// unit eigenvector by two steps of inverse iteration (T - theta I with a tiny shift).
void tridiagonal_top(const std::vector<double>& a, const std::vector<double>& b, double* theta, double* s_last) {
  const int k = (int)a.size();
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_above = [&](double x) {  // eigenvalues > x (Sturm sequence of T - x I)
    int neg = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      d = (a[i] - x) - (i > 0 ? bb / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++neg;
    }
    return k - neg;
  };
  for (int it = 0; it < 200 && hi - lo > 2e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_above(mid) >= 1) lo = mid; else hi = mid;
  }
  *theta = 0.5 * (lo + hi);
  if (k == 1) {
    *s_last = 1.0;
    return;
  }
  const double shift = *theta + 1e-13 * std::max(1.0, std::fabs(*theta));
  std::vector<double> x(k, 1.0), c(k), d(k), y(k);
  for (int rep = 0; rep < 3; ++rep) {  // solve (T - shift I) y = x (tridiagonal LU, no pivoting)
    for (int i = 0; i < k; ++i) {
      d[i] = a[i] - shift;
      y[i] = x[i];
    }
    for (int i = 1; i < k; ++i) {
      const double m = b[i - 1] / d[i - 1];
      d[i] -= m * b[i - 1];
      y[i] -= m * y[i - 1];
    }
    x[k - 1] = y[k - 1] / d[k - 1];
    for (int i = k - 2; i >= 0; --i) x[i] = (y[i] - b[i] * x[i + 1]) / d[i];
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double& v : x) v /= nrm;
  }
  *s_last = x[k - 1];
}

template <typename TV>
void lanczos_impl(chefsi_handle* h, const TV* v0, int steps, void* ws, const LzLayout& L, hipStream_t s,
                  std::vector<double>& a, std::vector<double>& b) {
  TV* vb[2] = {at<TV>(ws, L.v0), at<TV>(ws, L.v1)};
  double* w = at<double>(ws, L.w);
  double* part = at<double>(ws, L.partial);
  double* out = at<double>(ws, L.out);
  double* pin = h->pinned;
  auto read_scalar = [&]() {
    HIP_TRY(hipMemcpyAsync(pin, out, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return pin[0];
  };
  // v_1 = v0 / ||v0||
  HIP_TRY(launch_widen<TV>(v0, h->nd, w, s));
  HIP_TRY(launch_lanczos_norm<TV>(w, nullptr, 0.0, h->nd, part, out, s));
  const double n0 = std::sqrt(read_scalar());
  check(std::isfinite(n0) && n0 > 0.0, "the start vector must be finite and nonzero");
  HIP_TRY(launch_lanczos_scale<TV>(w, 1.0 / n0, h->nd, vb[0], s));
  int cur = 0;
  double beta = 0.0;
  for (int j = 0; j < steps; ++j) {
    const TV* v = vb[cur];
    TV* vprev = vb[cur ^ 1];
    apply_fused<TV, double, double>(h, v, nullptr, w, 1, 1.0, 0.0, 0.0, at<double>(ws, L.alpha), s);
    HIP_TRY(launch_lanczos_dot<TV>(w, v, j > 0 ? vprev : nullptr, beta, h->nd, part, out, s));
    const double alpha = read_scalar();
    HIP_TRY(launch_lanczos_norm<TV>(w, v, alpha, h->nd, part, out, s));
    beta = std::sqrt(read_scalar());
    if (!std::isfinite(alpha) || !std::isfinite(beta)) throw Error{CHEFSI_ERR_NONFINITE, "non-finite Lanczos coefficient"};
    a.push_back(alpha);
    b.push_back(beta);
    if (beta == 0.0) break;
    HIP_TRY(launch_lanczos_scale<TV>(w, 1.0 / beta, h->nd, vprev, s));  // v_{j+1} over v_{j-1}
    cur ^= 1;
  }
}

// ---------------------------------------------------------------------------
// Nonlocal forces.  Workspace: one gradient block (FP64, Nd x ns), the two coefficient
// blocks (np_tot x ns FP64), dV per projector column, occupations, forces.
// ---------------------------------------------------------------------------
struct FoLayout {
  size_t grad = 0, alpha = 0, beta = 0, dvc = 0, occ = 0, forces = 0, spart = 0, disp = 0, chiw = 0, nlsum = 0,
         total = 0;
};

FoLayout forces_layout(const chefsi_handle* h, int ns) {
  FoLayout L;
  const size_t np = (size_t)std::max(1, h->np_tot);
  size_t off = 0;
  L.grad = off;
  off += align256((size_t)h->nd * ns * 8);
  L.alpha = off;
  off += align256(np * ns * 8);
  L.beta = off;
  off += align256(np * ns * 8);
  L.dvc = off;
  off += align256(np * 8);
  L.occ = off;
  off += align256((size_t)ns * 8);
  L.forces = off;
  off += align256((size_t)std::max(1, h->n_atoms) * 3 * 8);
  L.spart = off;  // stress block sums (kVecBlocks x 6) and the six totals
  off += align256(((size_t)kVecBlocks * 6 + 8) * 8);
  // nonlocal stress: support-point displacements, the three displacement-weighted copies of
  // the projector values, and per-atom sums (energy + one n_atoms x 3 block per gradient
  // direction)
  const size_t nsupp = h->supp_idx_h.size(), nchi = h->chi_h.size();
  L.disp = off;
  off += align256(std::max<size_t>(1, 3 * nsupp) * 8);
  L.chiw = off;
  off += align256(std::max<size_t>(1, 3 * nchi) * 8);
  L.nlsum = off;
  off += align256((size_t)std::max(1, h->n_atoms) * 12 * 8);
  L.total = off;
  return L;
}

// Central first-derivative weights of order 2r: c_p = (-1)^(p+1) (r!)^2 / (p (r-p)! (r+p)!).
std::vector<double> first_derivative_weights(int r) {
  std::vector<double> c(r + 1, 0.0);
  auto fact = [](int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
  };
  for (int p = 1; p <= r; ++p)
    c[p] = ((p % 2) ? 1.0 : -1.0) * fact(r) * fact(r) / (p * fact(r - p) * fact(r + p));
  return c;
}

template <typename TV>
void forces_impl(chefsi_handle* h, const TV* X, int ns, const double* occ_host, void* ws, const FoLayout& L,
                 hipStream_t s, double* forces_host) {
  const std::vector<double> dvc(std::max(1, h->np_tot), h->dv);
  HIP_TRY(hipMemcpyAsync(at<double>(ws, L.dvc), dvc.data(), dvc.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<double>(ws, L.occ), occ_host, (size_t)ns * 8, hipMemcpyHostToDevice, s));
  double* alpha = at<double>(ws, L.alpha);
  double* beta = at<double>(ws, L.beta);
  double* grad = at<double>(ws, L.grad);
  const double* dv = at<double>(ws, L.dvc);
  HIP_TRY((launch_nl_project<TV, double>(nl_args<TV, double>(h, X, ns, h->chi64, dv, alpha), s)));
  const std::vector<double> c = first_derivative_weights(h->radius);
  for (int d = 0; d < 3; ++d) {
    GradArgs<TV> g{};
    g.x = X;
    g.out = grad;
    g.nd = h->nd;
    g.nx = h->n[0];
    g.ny = h->n[1];
    g.nz = h->n[2];
    g.dir = d;
    g.r = h->radius;
    g.periodic = h->bc[d] == 0 ? 1 : 0;
    for (int p = 0; p <= h->radius; ++p) g.c[p] = c[p];
    g.inv_h = 1.0 / h->h[d];
    HIP_TRY(launch_grad<TV>(g, ns, s));
    HIP_TRY((launch_nl_project<double, double>(nl_args<double, double>(h, grad, ns, h->chi64, dv, beta), s)));
    ForceArgs f{};
    f.alpha = alpha;
    f.beta = beta;
    f.occ = at<double>(ws, L.occ);
    f.gdv = h->gdv64;
    f.nproj = h->nproj;
    f.poff = h->poff;
    f.dv = h->dv;
    f.n_atoms = h->n_atoms;
    f.np_tot = h->np_tot;
    f.ns = ns;
    f.dir = d;
    f.forces = at<double>(ws, L.forces);
    HIP_TRY(launch_forces(f, s));
  }
  double* pin = nullptr;
  const size_t fb = (size_t)h->n_atoms * 3 * 8;
  HIP_TRY(hipHostMalloc((void**)&pin, fb, hipHostMallocDefault));
  hipError_t e = hipMemcpyAsync(pin, at<double>(ws, L.forces), fb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) std::memcpy(forces_host, pin, fb);
  (void)hipHostFree(pin);
  HIP_TRY(e);
}

// Nonlocal stress (see chefsi.h): alpha = dV chi^T psi, then per gradient direction a the
// gathers beta_ab = dV (chi d_b)^T (d psi / dx_a) and the per-atom sums
// -2 sum_k gamma_k sum_v g_v alpha beta_ab (force_kernel), and the energy's per-atom sums
// from beta = alpha; the atom sums are added on the host in atom order.
template <typename TV>
void nonlocal_stress_impl(chefsi_handle* h, const TV* X, int ns, const double* occ_host, const double* disp_host,
                          void* ws, const FoLayout& L, hipStream_t s, double* stress_host) {
  const int na = h->n_atoms;
  const size_t nsupp = h->supp_idx_h.size(), nchi = h->chi_h.size();
  const std::vector<double> dvc(std::max(1, h->np_tot), h->dv);
  HIP_TRY(hipMemcpyAsync(at<double>(ws, L.dvc), dvc.data(), dvc.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<double>(ws, L.occ), occ_host, (size_t)ns * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<double>(ws, L.disp), disp_host, 3 * nsupp * 8, hipMemcpyHostToDevice, s));
  double* chiw = at<double>(ws, L.chiw);
  ChiDispArgs cd{};
  cd.chi = h->chi64;
  cd.disp = at<double>(ws, L.disp);
  cd.supp_off = h->supp_off;
  cd.chi_off = h->chi_off;
  cd.nproj = h->nproj;
  cd.n_atoms = na;
  cd.nchi = (int64_t)nchi;
  cd.out = chiw;
  HIP_TRY(launch_chi_disp(cd, s));
  double* alpha = at<double>(ws, L.alpha);
  double* beta = at<double>(ws, L.beta);
  double* grad = at<double>(ws, L.grad);
  double* sums = at<double>(ws, L.nlsum);  // [0]: energy, [1 + a]: direction a; n_atoms x 3 each
  const double* dv = at<double>(ws, L.dvc);
  HIP_TRY((launch_nl_project<TV, double>(nl_args<TV, double>(h, X, ns, h->chi64, dv, alpha), s)));
  ForceArgs f{};
  f.alpha = alpha;
  f.occ = at<double>(ws, L.occ);
  f.gdv = h->gdv64;
  f.nproj = h->nproj;
  f.poff = h->poff;
  f.dv = h->dv;
  f.n_atoms = na;
  f.np_tot = h->np_tot;
  f.ns = ns;
  f.beta = alpha;
  f.dir = 0;
  f.forces = sums;
  HIP_TRY(launch_forces(f, s));
  const std::vector<double> c = first_derivative_weights(h->radius);
  for (int a = 0; a < 3; ++a) {
    GradArgs<TV> g{};
    g.x = X;
    g.out = grad;
    g.nd = h->nd;
    g.nx = h->n[0];
    g.ny = h->n[1];
    g.nz = h->n[2];
    g.dir = a;
    g.r = h->radius;
    g.periodic = h->bc[a] == 0 ? 1 : 0;
    for (int p = 0; p <= h->radius; ++p) g.c[p] = c[p];
    g.inv_h = 1.0 / h->h[a];
    HIP_TRY(launch_grad<TV>(g, ns, s));
    for (int b = 0; b < 3; ++b) {
      HIP_TRY((launch_nl_project<double, double>(
          nl_args<double, double>(h, grad, ns, chiw + (size_t)b * nchi, dv, beta), s)));
      f.beta = beta;
      f.dir = b;
      f.forces = sums + (size_t)(1 + a) * na * 3;
      HIP_TRY(launch_forces(f, s));
    }
  }
  const size_t nb = (size_t)na * 12 * 8;
  double* pin = nullptr;
  HIP_TRY(hipHostMalloc((void**)&pin, nb, hipHostMallocDefault));
  hipError_t e = hipMemcpyAsync(pin, sums, nb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  std::vector<double> hs;
  if (e == hipSuccess) hs.assign(pin, pin + (size_t)na * 12);
  (void)hipHostFree(pin);
  HIP_TRY(e);
  // energy: force_kernel gave -2 sum gamma g alpha^2 per atom (component 0)
  double e_nl = 0.0;
  for (int J = 0; J < na; ++J) e_nl += -0.5 * hs[(size_t)J * 3];
  const double omega = (double)h->nd * h->dv;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double t = 0.0;  // -2 sum g gamma alpha beta_ab
      for (int J = 0; J < na; ++J) t += hs[(size_t)(1 + a) * na * 3 + (size_t)J * 3 + b];
      stress_host[a * 3 + b] = -((a == b ? e_nl : 0.0) - t) / omega;
    }
}

template <typename TV>
void kinetic_stress_impl(chefsi_handle* h, const TV* X, int ns, const double* occ_host, void* ws, const FoLayout& L,
                         hipStream_t s, double* stress_host) {
  HIP_TRY(hipMemcpyAsync(at<double>(ws, L.occ), occ_host, (size_t)ns * 8, hipMemcpyHostToDevice, s));
  const std::vector<double> c = first_derivative_weights(h->radius);
  StressArgs<TV> a{};
  a.x = X;
  a.occ = at<double>(ws, L.occ);
  a.nd = h->nd;
  a.ns = ns;
  a.nx = h->n[0];
  a.ny = h->n[1];
  a.nz = h->n[2];
  a.r = h->radius;
  for (int d = 0; d < 3; ++d) {
    a.periodic[d] = h->bc[d] == 0 ? 1 : 0;
    a.inv_h[d] = 1.0 / h->h[d];
  }
  for (int p = 0; p <= h->radius; ++p) a.c[p] = c[p];
  a.partial = at<double>(ws, L.spart);
  a.out = a.partial + (size_t)kVecBlocks * 6;
  HIP_TRY(launch_stress_sums<TV>(a, s));
  double* pin = h->pinned;  // max_ns + 8 doubles; six needed
  double sums[6];
  HIP_TRY(hipMemcpyAsync(pin, a.out, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(sums, pin, sizeof(sums));
  // sigma_ab = -(dV / Omega) sum = -(1 / Nd) sum, Omega = Nd dV
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    const double v = -sums[k] / (double)h->nd;
    stress_host[ia[k] * 3 + ib[k]] = v;
    stress_host[ib[k] * 3 + ia[k]] = v;
  }
}

}  // namespace

extern "C" {

int chefsi_kinetic_stress(chefsi_handle_t* h, const void* X, int32_t ns, const double* occ_host, void* ws,
                          size_t ws_bytes, void* stream, double* stress_host) {
  return guarded(h, [&] {
    check(X != nullptr && occ_host != nullptr && stress_host != nullptr && ws != nullptr,
          "X, occ, stress and ws must not be NULL");
    check_ns(h, ns);
    for (int i = 0; i < ns; ++i) check(std::isfinite(occ_host[i]), "occupations must be finite");
    const FoLayout L = forces_layout(h, ns);
    if (ws_bytes < L.total) throw Error{CHEFSI_ERR_WORKSPACE, "workspace smaller than chefsi_forces_workspace_bytes"};
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64)
      kinetic_stress_impl<double>(h, (const double*)X, ns, occ_host, ws, L, s, stress_host);
    else
      kinetic_stress_impl<float>(h, (const float*)X, ns, occ_host, ws, L, s, stress_host);
  });
}

int chefsi_nonlocal_stress(chefsi_handle_t* h, const void* X, int32_t ns, const double* occ_host,
                           const double* disp_host, void* ws, size_t ws_bytes, void* stream, double* stress_host) {
  return guarded(h, [&] {
    check(X != nullptr && occ_host != nullptr && stress_host != nullptr, "X, occ and stress must not be NULL");
    check_ns(h, ns);
    for (int i = 0; i < ns; ++i) check(std::isfinite(occ_host[i]), "occupations must be finite");
    if (h->n_atoms == 0 || h->np_tot == 0) {
      std::fill(stress_host, stress_host + 9, 0.0);
      return;
    }
    check(disp_host != nullptr, "disp must not be NULL when there are projectors");
    const size_t nsupp = h->supp_idx_h.size();
    for (size_t i = 0; i < 3 * nsupp; ++i) check(std::isfinite(disp_host[i]), "displacements must be finite");
    check(ws != nullptr, "ws is NULL");
    const FoLayout L = forces_layout(h, ns);
    if (ws_bytes < L.total) throw Error{CHEFSI_ERR_WORKSPACE, "workspace smaller than chefsi_forces_workspace_bytes"};
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64)
      nonlocal_stress_impl<double>(h, (const double*)X, ns, occ_host, disp_host, ws, L, s, stress_host);
    else
      nonlocal_stress_impl<float>(h, (const float*)X, ns, occ_host, disp_host, ws, L, s, stress_host);
  });
}

int chefsi_forces_workspace_bytes(const chefsi_handle_t* hc, int32_t ns, size_t* bytes) {
  chefsi_handle* h = const_cast<chefsi_handle*>(hc);
  return guarded(h, [&] {
    check(bytes != nullptr, "bytes is NULL");
    check_ns(h, ns);
    *bytes = forces_layout(h, ns).total;
  });
}

int chefsi_nonlocal_forces(chefsi_handle_t* h, const void* X, int32_t ns, const double* occ_host, void* ws,
                           size_t ws_bytes, void* stream, double* forces_host) {
  return guarded(h, [&] {
    check(X != nullptr && occ_host != nullptr && forces_host != nullptr, "X, occ and forces must not be NULL");
    check_ns(h, ns);
    for (int i = 0; i < ns; ++i) check(std::isfinite(occ_host[i]), "occupations must be finite");
    if (h->n_atoms == 0 || h->np_tot == 0) {
      std::fill(forces_host, forces_host + 3 * (size_t)h->n_atoms, 0.0);
      return;
    }
    check(ws != nullptr, "ws is NULL");
    const FoLayout L = forces_layout(h, ns);
    if (ws_bytes < L.total) throw Error{CHEFSI_ERR_WORKSPACE, "workspace smaller than chefsi_forces_workspace_bytes"};
    hipStream_t s = (hipStream_t)stream;
    if (h->precision == CHEFSI_FP64)
      forces_impl<double>(h, (const double*)X, ns, occ_host, ws, L, s, forces_host);
    else
      forces_impl<float>(h, (const float*)X, ns, occ_host, ws, L, s, forces_host);
  });
}

int chefsi_lanczos_workspace_bytes(const chefsi_handle_t* hc, size_t* bytes) {
  chefsi_handle* h = const_cast<chefsi_handle*>(hc);
  return guarded(h, [&] {
    check(bytes != nullptr, "bytes is NULL");
    *bytes = lanczos_layout(h).total;
  });
}

int chefsi_lanczos_bound(chefsi_handle_t* h, const void* v0, int32_t steps, void* ws, size_t ws_bytes, void* stream,
                         double* lam_nd, double* theta, double* alpha_host, double* beta_host) {
  return guarded(h, [&] {
    check(v0 != nullptr && ws != nullptr, "v0 and ws must be device buffers");
    check(steps >= 1 && steps <= 1000, "steps must be in 1..1000");
    check(lam_nd != nullptr, "lam_nd is NULL");
    const LzLayout L = lanczos_layout(h);
    if (ws_bytes < L.total) throw Error{CHEFSI_ERR_WORKSPACE, "workspace smaller than chefsi_lanczos_workspace_bytes"};
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> a, b;
    if (h->precision == CHEFSI_FP64)
      lanczos_impl<double>(h, (const double*)v0, steps, ws, L, s, a, b);
    else
      lanczos_impl<float>(h, (const float*)v0, steps, ws, L, s, a, b);
    double th = 0.0, sl = 0.0;
    tridiagonal_top(a, b, &th, &sl);
    *lam_nd = th + std::fabs(b.back() * sl);
    if (theta) *theta = th;
    for (size_t i = 0; i < a.size(); ++i) {
      if (alpha_host) alpha_host[i] = a[i];
      if (beta_host) beta_host[i] = b[i];
    }
    for (size_t i = a.size(); i < (size_t)steps; ++i) {  // stopped early (invariant subspace)
      if (alpha_host) alpha_host[i] = 0.0;
      if (beta_host) beta_host[i] = 0.0;
    }
  });
}

int chefsi_set_stencil_tiling(chefsi_handle_t* h, int32_t rows_per_thread, int32_t row_groups) {
  return guarded(h, [&] {
    check(rows_per_thread >= 0 && rows_per_thread <= 4 && row_groups >= 0, "tiling parameters out of range");
    check((rows_per_thread == 0) == (row_groups == 0), "give both tiling parameters, or neither");
    const int eb = h->precision == CHEFSI_FP64 ? 8 : 4;
    const HxPlan p = plan_hx(h->n[0], h->n[1], h->n[2], 1, h->radius, eb, rows_per_thread, row_groups);
    check(p.ok, "the requested stencil tiling does not fit this grid");
    if (h->np_tot > 0)
      build_hx_records(h, p);
    else
      h->hx_plan = p;
  });
}

// Average time of one filter-form launch sequence (projector gather, stencil pass with the
// three-term update, scatter pass) on the first ns columns of X, written into the workspace
// block (X is not modified).
extern "C++" {
template <typename T>
static float time_filter_launch(chefsi_handle* h, const T* X, T* B, int ns, T* alpha, hipStream_t s,
                                hipEvent_t e0, hipEvent_t e1) {
  constexpr int kWarm = 1, kRuns = 3;
  for (int i = 0; i < kWarm; ++i) apply_fused<T, T, T>(h, X, B, B, ns, 0.5, 0.25, -0.5, alpha, s, false, true);
  HIP_TRY(hipEventRecord(e0, s));
  for (int i = 0; i < kRuns; ++i) apply_fused<T, T, T>(h, X, B, B, ns, 0.5, 0.25, -0.5, alpha, s, true, true);
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  return ms / kRuns;
}
}  // extern "C++"

// Switch the projector route of a handle with projectors (mode 4: records in the stencil
// pass, 0: band pass).  The band tables are built before anything else changes, so a
// route that cannot be built (a point in more than kBandMaxSlots projector supports, or
// records whose LDS does not fit the current tiling) throws and leaves the handle on its
// current route.
static void set_projector_route(chefsi_handle* h, int mode) {
  if (mode == 0) {
    build_band_tables(h);
    h->rec_max = 0;
    build_hx_records(h, h->hx_plan);
    build_scatter_records(h);
  } else {
    check(hx_records_fit(h, h->hx_plan), "too many projectors for the stencil pass (alpha row does not fit in LDS)");
    h->rec_max = mode;
    build_hx_records(h, h->hx_plan);
    build_scatter_records(h);
    free_band_tables(h);
  }
}

int chefsi_autotune(chefsi_handle_t* h, const void* X, int32_t ns, void* ws, size_t ws_bytes, void* stream,
                    int32_t* choice) {
  return guarded(h, [&] {
    check(X != nullptr, "X is NULL");
    check_ns(h, ns);
    WsLayout L;
    check_ws(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    const int nt = std::min(ns, 1024);  // orbitals timed: the per-orbital work is the same for all
    const int eb = h->precision == CHEFSI_FP64 ? 8 : 4;
    const int nx = h->n[0], ny = h->n[1];
    // candidate tilings: every row count per thread and row-group count the planner accepts,
    // tall tiles only (at least r + 1 rows, or the whole y extent)
    std::vector<HxPlan> cands;
    for (int py = 1; py <= 4; ++py)
      for (int nyg = 1; nx * nyg <= hx_max_threads(py); ++nyg) {
        if (py * nyg < std::min(h->radius + 1, ny) || py * nyg > ny + 2 * h->radius) continue;
        const HxPlan p = plan_hx(nx, ny, h->n[2], 1, h->radius, eb, py, nyg);
        if (p.ok) cands.push_back(p);
      }
    check(!cands.empty(), "no stencil tiling fits this grid");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct Events {
      hipEvent_t a, b;
      ~Events() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } ev{e0, e1};
    const bool prof = h->prof_on;
    h->prof_on = false;
    float best = 1e30f;
    int best_mode = h->rec_max, best_c = 0;
    const int modes[2] = {4, 0};
    for (int mode : modes) {
      if (h->np_tot == 0 && mode == 0) continue;
      if (h->rec_max != mode) {
        if (mode > 0)  // switch on the first tiling whose records fit (any tiling serves the band route)
          for (const HxPlan& c : cands)
            if (hx_records_fit(h, c)) {
              h->hx_plan = c;
              break;
            }
        try {
          set_projector_route(h, mode);
        } catch (const Error& e) {
          if (e.status == CHEFSI_ERR_INVALID_ARG) continue;  // this route cannot serve this handle
          throw;
        }
      }
      for (size_t c = 0; c < cands.size(); ++c) {
        if (h->np_tot > 0 && mode > 0 && !hx_records_fit(h, cands[c])) continue;  // tile too tall for the records
        if (h->np_tot > 0)
          build_hx_records(h, cands[c]);
        else
          h->hx_plan = cands[c];
        float ms;
        if (h->precision == CHEFSI_FP64)
          ms = time_filter_launch<double>(h, (const double*)X, at<double>(ws, L.bufB), nt, at<double>(ws, L.alpha),
                                          s, e0, e1);
        else
          ms = time_filter_launch<float>(h, (const float*)X, at<float>(ws, L.bufB), nt, at<float>(ws, L.alpha), s,
                                         e0, e1);
        if (ms < best) {
          best = ms;
          best_mode = mode;
          best_c = (int)c;
        }
      }
    }
    h->prof_on = prof;
    check(best < 1e30f, "no stencil tiling fits the projector records of this handle");
    h->hx_plan = cands[best_c];  // a route switch builds its records for the chosen tiling
    if (h->rec_max != best_mode) set_projector_route(h, best_mode);
    if (h->np_tot > 0)
      build_hx_records(h, cands[best_c]);
    else
      h->hx_plan = cands[best_c];
    if (choice) {
      choice[0] = cands[best_c].py;
      choice[1] = cands[best_c].nyg;
      choice[2] = best_mode > 0 ? 1 : 0;
    }
  });
}

int chefsi_set_projector_pass(chefsi_handle_t* h, int32_t in_stencil) {
  return guarded(h, [&] {
    check(in_stencil == 0 || in_stencil == 1, "in_stencil must be 0 or 1");
    const int want = in_stencil ? 4 : 0;
    if (want == h->rec_max || h->np_tot == 0) {
      h->rec_max = want;
      return;
    }
    set_projector_route(h, want);
  });
}

int chefsi_get_stencil_tiling(const chefsi_handle_t* hc, int32_t* tiling) {
  chefsi_handle* h = const_cast<chefsi_handle*>(hc);
  return guarded(h, [&] {
    check(tiling != nullptr, "tiling is NULL");
    tiling[0] = h->hx_plan.py;
    tiling[1] = h->hx_plan.nyg;
    tiling[2] = h->hx_plan.ty;
    tiling[3] = h->hx_plan.kh;
  });
}

int chefsi_handle_bytes(const chefsi_handle_t* h, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return CHEFSI_ERR_INVALID_ARG;
  *bytes = h->device_bytes;
  return CHEFSI_OK;
}

int chefsi_profile_enable(chefsi_handle_t* h, int32_t on) {
  return guarded(h, [&] { h->prof_on = on != 0; });
}

int chefsi_profile_reset(chefsi_handle_t* h) {
  return guarded(h, [&] {
    prof_collect(h);
    for (int i = 0; i < kNumProf; ++i) {
      h->prof_ms[i] = 0.0;
      h->prof_n[i] = 0;
    }
  });
}

int chefsi_profile_read(chefsi_handle_t* h, int32_t kernel_id, double* total_ms, int64_t* launches) {
  return guarded(h, [&] {
    check(kernel_id >= 0 && kernel_id < kNumProf, "kernel_id out of range");
    prof_collect(h);
    if (total_ms) *total_ms = h->prof_ms[kernel_id];
    if (launches) *launches = h->prof_n[kernel_id];
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// CheFSI at a Bloch wavevector (complex FP64; Sec. 2: every Brillouin-zone sample other
// than Gamma runs in complex double precision).  H_k = T_k + Veff + V_nl,k with
// Bloch-phased FD ghosts and Bloch-summed projectors; the step is Alg. 1 with conjugate
// transposes: Hs = X~^H H X~, Ms = X~^H X~ (rocBLAS zgemm), Ms = U^H U, C = U^-H Hs U^-1,
// C = W D W^H (rocSOLVER zheevd), Z = U^-1 W, X = X~ Z.
// ---------------------------------------------------------------------------
struct chefsi_kpoint {
  int device = 0;
  int n[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  int bc[3] = {0, 0, 0};
  int radius = 6;
  int64_t nd = 0;
  int max_ns = 0;
  double kvec[3] = {0, 0, 0};
  std::vector<double> w;
  int n_atoms = 0, np_tot = 0, n_pts = 0;
  double* veff = nullptr;
  double* gdv = nullptr;
  // band-pass tables (regions of touched points, complex chi~; the gather table conjugated)
  int nreg = 0;
  int *reg_pt = nullptr, *pt_idx = nullptr, *pt_ent = nullptr, *ent_ls = nullptr, *reg_slot = nullptr,
      *slot_q = nullptr, *slot_ent = nullptr, *gent_loc = nullptr, *q_slot_ptr = nullptr, *q_slot = nullptr;
  double2 *ent_chi = nullptr, *gent_chi = nullptr, *partial = nullptr;
  double* pinned = nullptr;
  rocblas_handle blas = nullptr;
  std::map<int, size_t> solver_ws_cache;
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<EventPair> ev_pending;
  double prof_ms[kNumProf] = {0};
  int64_t prof_n[kNumProf] = {0};
  std::string last_error;
};

namespace {

struct ZLayout {
  size_t bufB = 0, alpha = 0, hs = 0, ms = 0, d = 0, e = 0, info = 0, partial = 0, solver = 0, total = 0,
         solver_bytes = 0;
  BlasGram kg;  // K chunks of the projection (same split rule as the real FP64 Gram)
};

size_t zsolver_workspace(chefsi_kpoint* h, int ns) {
  auto it = h->solver_ws_cache.find(ns);
  if (it != h->solver_ws_cache.end()) return it->second;
  const rocblas_double_complex one(1.0, 0.0);
  size_t best = 0, sz = 0;
  auto query = [&](auto&& call) {
    BLAS_TRY(rocblas_start_device_memory_size_query(h->blas));
    call();
    BLAS_TRY(rocblas_stop_device_memory_size_query(h->blas, &sz));
    best = std::max(best, sz);
  };
  const rocblas_int ld = (rocblas_int)h->nd;
  query([&] { rocsolver_zpotrf(h->blas, rocblas_fill_upper, ns, nullptr, ns, nullptr); });
  query([&] {
    rocblas_ztrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_conjugate_transpose,
                  rocblas_diagonal_non_unit, ns, ns, &one, nullptr, ns, nullptr, ns);
  });
  query([&] {
    rocblas_ztrsm(h->blas, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none, rocblas_diagonal_non_unit,
                  ns, ns, &one, nullptr, ns, nullptr, ns);
  });
  query([&] {
    rocblas_ztrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none, rocblas_diagonal_non_unit,
                  ns, ns, &one, nullptr, ns, nullptr, ns);
  });
  query([&] {
    rocsolver_zheevd(h->blas, rocblas_evect_original, rocblas_fill_upper, ns, nullptr, ns, nullptr, nullptr, nullptr);
  });
  const BlasGram kg = plan_blas_gram(h->nd, ns);
  for (int q = 0; q < kg.nblk; ++q) {
    const int m = kg.start[q + 1] - kg.start[q], n = ns - kg.start[q];
    query([&] {
      rocblas_zgemm_strided_batched(h->blas, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, n,
                                    (rocblas_int)kg.kc, &one, nullptr, ld, kg.kc, nullptr, ld, kg.kc, &one, nullptr,
                                    ns, (rocblas_stride)ns * ns, kg.splits);
    });
    if (kg.tail > 0)
      query([&] {
        rocblas_zgemm(h->blas, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, n,
                      (rocblas_int)kg.tail, &one, nullptr, ld, nullptr, ld, &one, nullptr, ns);
      });
  }
  const rocblas_int prow = (rocblas_int)std::max<int64_t>(1, std::min<int64_t>(h->nd, (((int64_t)1 << 31) - 1) / ns));
  query([&] {
    rocblas_zgemm(h->blas, rocblas_operation_none, rocblas_operation_none, prow, ns, ns, &one, nullptr, ld, nullptr,
                  ns, &one, nullptr, ld);
  });
  h->solver_ws_cache[ns] = best;
  return best;
}

ZLayout zlayout(chefsi_kpoint* h, int ns) {
  ZLayout L;
  size_t off = 0;
  L.bufB = off;
  off += align256((size_t)h->nd * ns * 16);
  L.alpha = off;
  off += align256((size_t)std::max(1, h->np_tot) * ns * 16);
  L.hs = off;
  off += align256((size_t)ns * ns * 16);
  L.ms = off;
  off += align256((size_t)ns * ns * 16);
  L.d = off;
  off += align256((size_t)ns * 8);
  L.e = off;
  off += align256((size_t)ns * 8);
  L.info = off;
  off += 256;
  L.kg = plan_blas_gram(h->nd, ns);
  L.partial = off;
  off += align256((size_t)L.kg.nparts * ns * ns * 16);
  L.solver = off;
  L.solver_bytes = zsolver_workspace(h, ns);
  off += align256(std::max<size_t>(L.solver_bytes, 256));
  L.total = off;
  return L;
}

template <typename T>
T* zat(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

template <typename T>
T* kupload(const T* src, size_t n) {
  T* d = nullptr;
  if (n == 0) return nullptr;
  if (hipMalloc(&d, n * sizeof(T)) != hipSuccess) throw Error{CHEFSI_ERR_OOM, "device allocation failed"};
  hipError_t e = hipMemcpy(d, src, n * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    throw Error{CHEFSI_ERR_HIP, std::string("upload: ") + hipGetErrorString(e)};
  }
  return d;
}

void krelease(chefsi_kpoint* h) {
  void* ptrs[] = {h->veff,     h->gdv,      h->reg_pt,   h->pt_idx,     h->pt_ent,   h->ent_ls, h->reg_slot,
                  h->slot_q,   h->slot_ent, h->gent_loc, h->q_slot_ptr, h->q_slot,   h->ent_chi, h->gent_chi,
                  h->partial};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& p : h->ev_pending) {
    (void)hipEventDestroy(p.b);
    (void)hipEventDestroy(p.e);
  }
  for (auto ev : h->ev_pool) (void)hipEventDestroy(ev);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->blas) rocblas_destroy_handle(h->blas);
}

// k-point kernel classes timed by chefsi_kpoint_profile_*
enum KProfId { KP_ZHX = 0, KP_BAND = 1, KP_GRAM = 2, KP_EIG = 3, KP_ROT = 4 };
using KProfScope = ProfScopeT<chefsi_kpoint>;

ZNbArgs zband_args(const chefsi_kpoint* h, double2* y, int ns, const double2* alpha, double sa) {
  ZNbArgs b{};
  b.y = y;
  b.nd = h->nd;
  b.ns = ns;
  b.nreg = h->nreg;
  b.reg_pt = h->reg_pt;
  b.pt_idx = h->pt_idx;
  b.pt_ent = h->pt_ent;
  b.ent_ls = h->ent_ls;
  b.ent_chi = h->ent_chi;
  b.reg_slot = h->reg_slot;
  b.slot_q = h->slot_q;
  b.slot_ent = h->slot_ent;
  b.gent_loc = h->gent_loc;
  b.gent_chi = h->gent_chi;
  b.alpha = alpha;
  b.sa = sa;
  b.partial = h->partial;
  return b;
}

// out = sa ((H_k x) - sc x) + sb prev: stencil + Veff + recurrence, then the band pass adds
// sa V_nl x at the touched points (coefficients alpha of x: formed first by a gather-only
// pass unless alpha_ready) and, when want_next, leaves the coefficients of out in alpha.
void zapply(chefsi_kpoint* h, const double2* x, const double2* prev, double2* out, int ns, double sa, double sc,
            double sb, double2* alpha, hipStream_t s, bool alpha_ready = false, bool want_next = false) {
  if (h->np_tot > 0 && !alpha_ready) {
    KProfScope ps(h, KP_BAND, s);
    HIP_TRY(launch_zband(zband_args(h, const_cast<double2*>(x), ns, alpha, 0.0), false, true, s));
    HIP_TRY(launch_zband_reduce(h->partial, h->q_slot_ptr, h->q_slot, h->gdv, h->np_tot, ns, alpha, s));
    ps.done();
  }
  ZHxArgs a{};
  a.x = x;
  a.prev = prev;
  a.out = out;
  a.veff = h->veff;
  a.r = h->radius;
  a.nd = h->nd;
  double sumh = 0.0;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = h->n[d];
    a.per[d] = h->bc[d] == 0;
    sumh += 1.0 / (h->h[d] * h->h[d]);
    const double th = h->bc[d] == 0 ? h->kvec[d] * h->n[d] * h->h[d] : 0.0;
    a.ph[d] = make_double2(std::cos(th), std::sin(th));
    for (int p = 0; p <= kMaxRadius; ++p) a.cw[d][p] = p <= h->radius ? -0.5 * h->w[p] / (h->h[d] * h->h[d]) : 0.0;
  }
  a.c0 = -0.5 * h->w[0] * sumh;
  a.sa = sa;
  a.sc = sc;
  a.sb = sb;
  {
    KProfScope ps(h, KP_ZHX, s);
    HIP_TRY(launch_zhx(a, ns, s));
    ps.done();
  }
  if (h->np_tot > 0) {
    KProfScope ps(h, KP_BAND, s);
    HIP_TRY(launch_zband(zband_args(h, out, ns, alpha, sa), true, want_next, s));
    if (want_next)
      HIP_TRY(launch_zband_reduce(h->partial, h->q_slot_ptr, h->q_slot, h->gdv, h->np_tot, ns, alpha, s));
    ps.done();
  }
}

template <typename F>
int kguarded(chefsi_kpoint* h, F&& f) {
  if (h == nullptr) return CHEFSI_ERR_INVALID_ARG;
  try {
    h->last_error.clear();
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) HIP_TRY(hipSetDevice(h->device));
    f();
    return CHEFSI_OK;
  } catch (const Error& e) {
    h->last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    h->last_error = "host allocation failed";
    return CHEFSI_ERR_OOM;
  } catch (...) {
    h->last_error = "unexpected exception";
    return CHEFSI_ERR_HIP;
  }
}

void kcheck_call(chefsi_kpoint* h, int ns, void* ws, size_t ws_bytes, ZLayout& L) {
  check(ns >= 1 && ns <= h->max_ns, "ns must satisfy 1 <= ns <= max_ns");
  check((int64_t)ns <= h->nd, "ns must not exceed Nd");
  L = zlayout(h, ns);
  if (ws == nullptr || ws_bytes < L.total)
    throw Error{CHEFSI_ERR_WORKSPACE, "workspace smaller than chefsi_kpoint_workspace_bytes(ns)"};
  check(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
}

}  // namespace

extern "C" {

int chefsi_kpoint_create(const chefsi_grid_t* grid, const double* veff_host, const chefsi_nonlocal_t* nl,
                         const int32_t* supp_img, const double* kvec, int32_t max_ns, chefsi_kpoint_t** out) {
  if (out == nullptr) return CHEFSI_ERR_INVALID_ARG;
  *out = nullptr;
  if (grid == nullptr || veff_host == nullptr || kvec == nullptr) return CHEFSI_ERR_INVALID_ARG;
  chefsi_kpoint* h = nullptr;
  try {
    h = new chefsi_kpoint();
  } catch (...) {
    return CHEFSI_ERR_OOM;
  }
  try {
    check(grid->fd_order >= 2 && grid->fd_order <= 12 && grid->fd_order % 2 == 0, "fd_order must be even, 2..12");
    h->radius = grid->fd_order / 2;
    int64_t nd = 1;
    for (int d = 0; d < 3; ++d) {
      check(grid->n[d] >= 1, "grid sizes must be >= 1");
      check(grid->bc[d] == 0 || grid->bc[d] == 1, "bc must be 0 (periodic) or 1 (Dirichlet)");
      check(std::isfinite(grid->h[d]) && grid->h[d] > 0.0, "grid spacing must be positive");
      check(std::isfinite(kvec[d]), "k must be finite");
      if (grid->bc[d] == 0) check(grid->n[d] >= h->radius, "periodic direction needs n >= fd_order/2");
      h->n[d] = grid->n[d];
      h->h[d] = grid->h[d];
      h->bc[d] = grid->bc[d];
      h->kvec[d] = kvec[d];
      nd *= grid->n[d];
    }
    check(nd < (int64_t)1 << 31, "Nd must be below 2^31");
    check(max_ns >= 1 && (int64_t)max_ns <= nd && max_ns <= 65535, "max_ns must satisfy 1 <= max_ns <= min(Nd, 65535)");
    {
      const ZTiling zt = plan_zhx(grid->n[0], grid->n[1], grid->n[2], 1, grid->fd_order / 2);
      check(grid->n[0] <= kZMaxThreads && zt.kh <= 4 && zt.lds_bytes <= 96 * 1024,
            "grid too wide in x for the complex stencil tiling (halo values per thread above four)");
    }
    h->nd = nd;
    h->max_ns = max_ns;
    h->w = fd_weights(grid->fd_order);
    const double dv = grid->h[0] * grid->h[1] * grid->h[2];
    std::vector<double> veff(veff_host, veff_host + nd);
    for (double v : veff) check(std::isfinite(v), "Veff must be finite");

    std::vector<int> soff, sidx, nproj, poff, cnt, cols;
    std::vector<int64_t> coff;
    std::vector<double2> chi, vals;
    std::vector<double> gdv;
    if (nl != nullptr && nl->n_atoms > 0) {
      check(nl->supp_ptr && nl->supp_idx && nl->nproj && nl->chi && nl->gamma && supp_img, "null projector array");
      const int na = nl->n_atoms;
      const int64_t nsupp = nl->supp_ptr[na];
      check(nl->supp_ptr[0] == 0 && nsupp >= 0 && nsupp < (int64_t)1 << 31, "bad supp_ptr");
      double kl[3];
      for (int d = 0; d < 3; ++d) kl[d] = grid->bc[d] == 0 ? kvec[d] * grid->n[d] * grid->h[d] : 0.0;
      soff.resize(na + 1);
      coff.resize(na);
      poff.resize(na);
      nproj.assign(nl->nproj, nl->nproj + na);
      int64_t c = 0;
      int p = 0;
      for (int J = 0; J < na; ++J) {
        check(nl->supp_ptr[J + 1] >= nl->supp_ptr[J], "supp_ptr must be non-decreasing");
        check(nproj[J] >= 1, "nproj must be >= 1");
        soff[J] = (int)nl->supp_ptr[J];
        coff[J] = c;
        poff[J] = p;
        const int64_t nj = nl->supp_ptr[J + 1] - nl->supp_ptr[J];
        for (int64_t s = 0; s < nj; ++s) {
          const int64_t i = nl->supp_idx[nl->supp_ptr[J] + s];
          check(i >= 0 && i < nd, "support index outside the grid");
          if (s > 0) check(i > nl->supp_idx[nl->supp_ptr[J] + s - 1], "support indices must increase");
        }
        c += nj * nproj[J];
        p += nproj[J];
      }
      check(p < (1 << 30) && c < ((int64_t)1 << 31), "too many projectors");
      soff[na] = (int)nsupp;
      h->n_atoms = na;
      h->np_tot = p;
      sidx.assign(nl->supp_idx, nl->supp_idx + nsupp);
      // Bloch-phased projector values: chi~ = chi * exp(i k.(m L)), m the image of the point
      chi.resize(c);
      for (int J = 0; J < na; ++J) {
        const int64_t nj = nl->supp_ptr[J + 1] - nl->supp_ptr[J];
        for (int64_t s = 0; s < nj; ++s) {
          const int64_t g = nl->supp_ptr[J] + s;
          double th = 0.0;
          for (int d = 0; d < 3; ++d) th += kl[d] * supp_img[3 * g + d];
          const double cr = std::cos(th), ci = std::sin(th);
          for (int a = 0; a < nproj[J]; ++a) {
            const double v = nl->chi[coff[J] + a * nj + s];
            check(std::isfinite(v), "chi must be finite");
            chi[coff[J] + a * nj + s] = make_double2(v * cr, v * ci);
          }
        }
      }
      gdv.resize(p);
      for (int q = 0; q < p; ++q) {
        check(std::isfinite(nl->gamma[q]), "gamma must be finite");
        gdv[q] = nl->gamma[q] * dv;
      }
      // point-major entries: grid points in increasing order, atoms in order
      cnt.assign(nd + 1, 0);
      for (int J = 0; J < na; ++J)
        for (int64_t s = nl->supp_ptr[J]; s < nl->supp_ptr[J + 1]; ++s) cnt[sidx[s] + 1] += nproj[J];
      for (int64_t i = 0; i < nd; ++i) cnt[i + 1] += cnt[i];
      const int64_t nent = cnt[nd];
      std::vector<int> fill(cnt.begin(), cnt.end() - 1);
      cols.resize(nent);
      vals.resize(nent);
      for (int J = 0; J < na; ++J) {
        const int64_t nj = nl->supp_ptr[J + 1] - nl->supp_ptr[J];
        for (int64_t s = 0; s < nj; ++s) {
          const int i = sidx[nl->supp_ptr[J] + s];
          for (int a = 0; a < nproj[J]; ++a) {
            const int pos = fill[i]++;
            cols[pos] = poff[J] + a;
            vals[pos] = chi[coff[J] + a * nj + s];
          }
        }
      }
      check(nent < ((int64_t)1 << 31), "too many projector entries");
    }

    HIP_TRY(hipGetDevice(&h->device));
    BLAS_TRY(rocblas_create_handle(&h->blas));
    BLAS_TRY(rocblas_set_atomics_mode(h->blas, rocblas_atomics_not_allowed));
    if (hipHostMalloc((void**)&h->pinned, (size_t)max_ns * sizeof(double) + 64, hipHostMallocDefault) != hipSuccess) {
      h->pinned = nullptr;
      throw Error{CHEFSI_ERR_OOM, "pinned host allocation failed"};
    }
    h->veff = kupload(veff.data(), veff.size());
    if (h->np_tot > 0) {
      // band-pass regions of the touched points (the real path's tables with chi~ values)
      const BandRegions R = band_regions(nd, cnt.data(), cols.data(), h->np_tot, kZBandMaxEnt);
      std::vector<double2> ent_chi(R.ent_src.size()), gent_chi(R.gent_src.size());
      for (size_t e = 0; e < ent_chi.size(); ++e) ent_chi[e] = vals[R.ent_src[e]];
      for (size_t e = 0; e < gent_chi.size(); ++e) {
        const double2 v = vals[R.gent_src[e]];
        gent_chi[e] = make_double2(v.x, -v.y);
      }
      h->nreg = (int)R.reg_pt.size() - 1;
      h->n_pts = (int)R.pt_idx.size();
      h->gdv = kupload(gdv.data(), gdv.size());
      h->reg_pt = kupload(R.reg_pt.data(), R.reg_pt.size());
      h->pt_idx = kupload(R.pt_idx.data(), R.pt_idx.size());
      h->pt_ent = kupload(R.pt_ent.data(), R.pt_ent.size());
      h->ent_ls = kupload(R.ent_ls.data(), R.ent_ls.size());
      h->ent_chi = kupload(ent_chi.data(), ent_chi.size());
      h->reg_slot = kupload(R.reg_slot.data(), R.reg_slot.size());
      h->slot_q = kupload(R.slot_q.data(), R.slot_q.size());
      h->slot_ent = kupload(R.slot_ent.data(), R.slot_ent.size());
      h->gent_loc = kupload(R.gent_loc.data(), R.gent_loc.size());
      h->gent_chi = kupload(gent_chi.data(), gent_chi.size());
      h->q_slot_ptr = kupload(R.q_slot_ptr.data(), R.q_slot_ptr.size());
      h->q_slot = kupload(R.q_slot.data(), R.q_slot.size());
      if (hipMalloc((void**)&h->partial, std::max<size_t>(1, R.slot_q.size()) * (size_t)max_ns * sizeof(double2)) !=
          hipSuccess) {
        h->partial = nullptr;
        throw Error{CHEFSI_ERR_OOM, "device allocation failed (band-pass partial sums)"};
      }
    }
    *out = h;
    return CHEFSI_OK;
  } catch (const Error& e) {
    krelease(h);
    delete h;
    return e.status;
  } catch (...) {
    krelease(h);
    delete h;
    return CHEFSI_ERR_OOM;
  }
}

void chefsi_kpoint_destroy(chefsi_kpoint_t* h) {
  if (h == nullptr) return;
  (void)hipSetDevice(h->device);
  krelease(h);
  delete h;
}

const char* chefsi_kpoint_last_error(const chefsi_kpoint_t* h) { return h ? h->last_error.c_str() : ""; }

int chefsi_kpoint_profile_enable(chefsi_kpoint_t* h, int32_t on) {
  return kguarded(h, [&] { h->prof_on = on != 0; });
}

int chefsi_kpoint_profile_reset(chefsi_kpoint_t* h) {
  return kguarded(h, [&] {
    prof_collect(h);
    for (int i = 0; i < kNumProf; ++i) {
      h->prof_ms[i] = 0.0;
      h->prof_n[i] = 0;
    }
  });
}

int chefsi_kpoint_profile_read(chefsi_kpoint_t* h, int32_t kernel_id, double* total_ms, int64_t* launches) {
  return kguarded(h, [&] {
    check(kernel_id >= 0 && kernel_id <= KP_ROT, "kernel_id out of range");
    prof_collect(h);
    if (total_ms) *total_ms = h->prof_ms[kernel_id];
    if (launches) *launches = h->prof_n[kernel_id];
  });
}

int chefsi_kpoint_workspace_bytes(chefsi_kpoint_t* h, int32_t ns, size_t* bytes) {
  return kguarded(h, [&] {
    check(bytes != nullptr, "null pointer");
    check(ns >= 1 && ns <= h->max_ns, "ns must satisfy 1 <= ns <= max_ns");
    *bytes = zlayout(h, ns).total;
  });
}

int chefsi_kpoint_apply_h(chefsi_kpoint_t* h, const void* X, void* Y, int32_t ns, void* ws, size_t ws_bytes,
                          void* stream) {
  return kguarded(h, [&] {
    check(X != nullptr && Y != nullptr, "null pointer");
    check(X != Y, "X and Y must not alias");
    ZLayout L;
    kcheck_call(h, ns, ws, ws_bytes, L);
    zapply(h, (const double2*)X, nullptr, (double2*)Y, ns, 1.0, 0.0, 0.0, zat<double2>(ws, L.alpha),
           (hipStream_t)stream);
  });
}

int chefsi_kpoint_step(chefsi_kpoint_t* h, void* X, int32_t ns, int32_t degree, double lam_lo, double lam_cut,
                       double lam_hi, void* ws, size_t ws_bytes, void* stream, double* ritz_host) {
  return kguarded(h, [&] {
    check(X != nullptr, "X is NULL");
    check(degree >= 1, "degree must be >= 1");
    check_bounds(lam_lo, lam_cut, lam_hi);
    ZLayout L;
    kcheck_call(h, ns, ws, ws_bytes, L);
    hipStream_t s = (hipStream_t)stream;
    double2* A = (double2*)X;
    double2* B = zat<double2>(ws, L.bufB);
    double2* alpha = zat<double2>(ws, L.alpha);
    double2* Hs = zat<double2>(ws, L.hs);
    double2* Ms = zat<double2>(ws, L.ms);
    double* D = zat<double>(ws, L.d);
    rocblas_int* info = zat<rocblas_int>(ws, L.info);
    // scaled Chebyshev filter (Alg. 1, Filtering), the same scalars as the real path
    const double c = 0.5 * (lam_hi + lam_cut);
    const double e = 0.5 * (lam_hi - lam_cut);
    const double s1 = e / (lam_lo - c);
    double sig = s1;
    // the projector coefficients of each output are left by its band pass for the next
    // application
    zapply(h, A, nullptr, B, ns, s1 / e, c, 0.0, alpha, s, false, true);
    double2* cur = B;
    double2* other = A;
    for (int k = 1; k < degree; ++k) {
      const double sig_next = 1.0 / (2.0 / s1 - sig);
      zapply(h, cur, other, other, ns, 2.0 * sig_next / e, c, -sig * sig_next, alpha, s, true, true);
      std::swap(cur, other);
      sig = sig_next;
    }
    double2* Xf = cur;
    double2* Yf = other;
    zapply(h, Xf, nullptr, Yf, ns, 1.0, 0.0, 0.0, alpha, s, true, false);  // Y~ = H X~
    // projection (upper triangles made Hermitian)
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    const rocblas_int ld = (rocblas_int)h->nd;
    BLAS_TRY(rocblas_set_stream(h->blas, s));
    BLAS_TRY(rocblas_set_workspace(h->blas, zat<void>(ws, L.solver), std::max<size_t>(L.solver_bytes, 256)));
    auto zc = [](const double2* p) { return reinterpret_cast<const rocblas_double_complex*>(p); };
    auto zm = [](double2* p) { return reinterpret_cast<rocblas_double_complex*>(p); };
    // split-K: K chunks as one strided batch of products, partials summed in a fixed order
    double2* part = zat<double2>(ws, L.partial);
    const BlasGram& kg = L.kg;
    // upper triangle only, by the real path's column blocks: block row q of every partial
    // against columns [start_q, ns)
    auto gram = [&](const double2* A, const double2* Bm, double2* C) {
      for (int q = 0; q < kg.nblk; ++q) {
        const int r0 = kg.start[q], m = kg.start[q + 1] - r0, n = ns - r0;
        const double2* Aq = A + (size_t)r0 * h->nd;
        const double2* Bq = Bm + (size_t)r0 * h->nd;
        double2* Pq = part + r0 + (size_t)r0 * ns;
        BLAS_TRY(rocblas_zgemm_strided_batched(h->blas, rocblas_operation_conjugate_transpose,
                                               rocblas_operation_none, m, n, (rocblas_int)kg.kc, &one, zc(Aq), ld,
                                               kg.kc, zc(Bq), ld, kg.kc, &zero, zm(Pq), ns, (rocblas_stride)ns * ns,
                                               kg.splits));
        if (kg.tail > 0) {
          const int64_t k0 = kg.kc * kg.splits;
          BLAS_TRY(rocblas_zgemm(h->blas, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, n,
                                 (rocblas_int)kg.tail, &one, zc(Aq + k0), ld, zc(Bq + k0), ld, &zero,
                                 zm(Pq + (size_t)kg.splits * ns * ns), ns));
        }
      }
      HIP_TRY(launch_zsum_partials(part, kg.nparts, ns, C, s));
    };
    {
      KProfScope ps(h, KP_GRAM, s);
      gram(Xf, Yf, Hs);
      gram(Xf, Xf, Ms);
      ps.done();
    }
    // Hermitian-definite eigenproblem (Alg. 1, Diagonalization)
    KProfScope pe(h, KP_EIG, s);
    BLAS_TRY(rocsolver_zpotrf(h->blas, rocblas_fill_upper, ns, zm(Ms), ns, info));
    BLAS_TRY(rocblas_ztrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_conjugate_transpose,
                           rocblas_diagonal_non_unit, ns, ns, &one, zc(Ms), ns, zm(Hs), ns));
    BLAS_TRY(rocblas_ztrsm(h->blas, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                           rocblas_diagonal_non_unit, ns, ns, &one, zc(Ms), ns, zm(Hs), ns));
    BLAS_TRY(rocsolver_zheevd(h->blas, rocblas_evect_original, rocblas_fill_upper, ns, zm(Hs), ns, D,
                              zat<double>(ws, L.e), info + 1));
    BLAS_TRY(rocblas_ztrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                           rocblas_diagonal_non_unit, ns, ns, &one, zc(Ms), ns, zm(Hs), ns));
    pe.done();
    KProfScope pr(h, KP_ROT, s);
    // rotation (Alg. 1, Rotation): X = X~ Z into the buffer Y~ held, in row panels of fewer
    // than 2^31 output elements each (blocks of any size)
    const int64_t prow = std::max<int64_t>(1, std::min<int64_t>(h->nd, (((int64_t)1 << 31) - 1) / ns));
    for (int64_t r0 = 0; r0 < h->nd; r0 += prow) {
      const rocblas_int m = (rocblas_int)std::min<int64_t>(prow, h->nd - r0);
      BLAS_TRY(rocblas_zgemm(h->blas, rocblas_operation_none, rocblas_operation_none, m, ns, ns, &one, zc(Xf + r0),
                             ld, zc(Hs), ns, &zero, zm(Yf + r0), ld));
    }
    if (Yf != A) HIP_TRY(hipMemcpyAsync(A, Yf, (size_t)h->nd * ns * 16, hipMemcpyDeviceToDevice, s));
    pr.done();
    double* d = h->pinned;
    rocblas_int* inf = reinterpret_cast<rocblas_int*>(h->pinned + h->max_ns);
    HIP_TRY(hipMemcpyAsync(d, D, (size_t)ns * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(inf, info, 2 * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (inf[0] > 0) throw Error{CHEFSI_ERR_NOT_POSDEF, "Cholesky of the overlap matrix failed"};
    if (inf[1] > 0) throw Error{CHEFSI_ERR_EIG, "dense eigensolver did not converge"};
    for (int i = 0; i < ns; ++i)
      if (!std::isfinite(d[i])) throw Error{CHEFSI_ERR_NONFINITE, "non-finite Ritz value"};
    if (ritz_host) std::memcpy(ritz_host, d, (size_t)ns * 8);
  });
}

}  // extern "C"
