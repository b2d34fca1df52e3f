// MI355X batched stiff-chemistry integrator: kernels and the C ABI of chem.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/chem.h"
#include "chem_adjoint.hpp"
#include "chem_wg.hpp"
#include "chem_seulex.hpp"
#include "chem_cell.hpp"

using namespace chem;

// ===================================================================== kernels
namespace {

constexpr int MAX_WPB = 8;

__device__ inline void stage_blob(uint8_t* lds, const uint8_t* blob, int bytes) {
  const uint4* src = (const uint4*)blob;
  uint4* dst = (uint4*)lds;
  for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

template <int NP>
constexpr int max_threads() {
  return NP <= 16 ? 64 * MAX_WPB : 256;
}

template <int NP, bool PROF>
__global__ __launch_bounds__(max_threads<NP>()) void k_integrate(IntArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  stage_blob(lds, a.blob, a.d.lds_bytes);
  const MechView m = make_view(lds, a);
  const int wv = threadIdx.x / WAVE;
  const CellWs w = make_ws((double*)(lds + a.d.lds_bytes) + (size_t)wv * a.cell_doubles, a.d);
  // one call site: a persistent wave pulls cells from the queue until it is
  // drained, a plain wave handles the one cell of its slot
  int64_t idx;
  if (a.queue) {
    int v = 0;
    if (lane_id() == 0) v = atomicAdd(a.queue, 1);
    idx = uniform_int(__shfl(v, 0));
  } else {
    idx = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
  }
  const int64_t lim = a.nactive ? (int64_t)*a.nactive : a.ncells;
  while (idx < lim) {
    const int64_t c = a.order ? (int64_t)a.order[idx] : idx;
    integrate_cell<NP, PROF>(m, w, a, c);
    if (!a.queue) break;
    int v = 0;
    if (lane_id() == 0) v = atomicAdd(a.queue, 1);
    idx = uniform_int(__shfl(v, 0));
  }
}

// The Rosenbrock integrator with Jacobian slots shared by the workgroup's
// waves (LDS: blob, each wave's workspace without a Jacobian block, slot
// flags, slots).  Up to eight cells per workgroup and CU instead of the four
// whose private Jacobian blocks fit, so each SIMD runs two waves.
template <int NP, bool PROF>
__global__ __launch_bounds__(512) void k_integrate_pool(IntArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int nw = blockDim.x / WAVE;
  int* flags = (int*)(lds + a.d.lds_bytes + (size_t)nw * a.cell_doubles * sizeof(double));
  double* slots = (double*)((uint8_t*)flags + 64);
  if (threadIdx.x < (unsigned)a.pool_slots) flags[threadIdx.x] = 0;
  stage_blob(lds, a.blob, a.d.lds_bytes);  // ends with a workgroup barrier
  const MechView m = make_view(lds, a);
  const int wv = threadIdx.x / WAVE;
  const CellWs w = make_ws((double*)(lds + a.d.lds_bytes) + (size_t)wv * a.cell_doubles, a.d, false);
  const SlotPool pool{flags, slots, a.pool_slots, a.d.N * a.d.S};
  int64_t idx;
  if (a.queue) {
    int v = 0;
    if (lane_id() == 0) v = atomicAdd(a.queue, 1);
    idx = uniform_int(__shfl(v, 0));
  } else {
    idx = (int64_t)blockIdx.x * nw + wv;
  }
  const int64_t lim = a.nactive ? (int64_t)*a.nactive : a.ncells;
  while (idx < lim) {
    const int64_t c = a.order ? (int64_t)a.order[idx] : idx;
    integrate_cell<NP, PROF>(m, w, a, c, &pool);
    if (!a.queue) break;
    int v = 0;
    if (lane_id() == 0) v = atomicAdd(a.queue, 1);
    idx = uniform_int(__shfl(v, 0));
  }
}

// The same launch structure with the Seulex-family integrator.
template <int NP, bool PROF>
__global__ __launch_bounds__(max_threads<NP>()) void k_integrate_sx(IntArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  stage_blob(lds, a.blob, a.d.lds_bytes);
  const MechView m = make_view(lds, a);
  const int wv = threadIdx.x / WAVE;
  const CellWs w = make_ws((double*)(lds + a.d.lds_bytes) + (size_t)wv * a.cell_doubles, a.d);
  int64_t idx;
  if (a.queue) {
    int v = 0;
    if (lane_id() == 0) v = atomicAdd(a.queue, 1);
    idx = uniform_int(__shfl(v, 0));
  } else {
    idx = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
  }
  const int64_t lim = a.nactive ? (int64_t)*a.nactive : a.ncells;
  while (idx < lim) {
    const int64_t c = a.order ? (int64_t)a.order[idx] : idx;
    integrate_cell_sx<NP, PROF>(m, w, a, c);
    if (!a.queue) break;
    int v = 0;
    if (lane_id() == 0) v = atomicAdd(a.queue, 1);
    idx = uniform_int(__shfl(v, 0));
  }
}

__global__ void k_reset(int* q, unsigned long long* failed) {
  if (threadIdx.x == 0) {
    if (q) *q = 0;
    if (failed) *failed = 0ull;
  }
}

template <int NP>
__global__ __launch_bounds__(max_threads<NP>()) void k_rhs_jac(IntArgs a, const double* st, double* f, double* J) {
  extern __shared__ __align__(16) uint8_t lds[];
  stage_blob(lds, a.blob, a.d.lds_bytes);
  const MechView m = make_view(lds, a);
  const int wv = threadIdx.x / WAVE;
  const CellWs w = make_ws((double*)(lds + a.d.lds_bytes) + (size_t)wv * a.cell_doubles, a.d);
  const int64_t c = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
  if (c >= a.ncells) return;
  const int lane = lane_id();
  const int N = m.d.N;
  if (lane == 0) {
    w.C[m.d.K] = 1.0;
    w.g[m.d.K] = 0.0;
    w.hR[m.d.K] = 0.0;
  }
  wsync();
  const double y = lane < N ? st[(int64_t)lane * a.ld + c] : 0.0;
  double row[NP];
  double fv;
  if (J) {
    fv = jac_pass<NP>(m, w, y, a.p, lane, row);
    if (lane < N)
      for (int j = 0; j < N; ++j) J[((size_t)c * N + lane) * N + j] = w.J[lane * m.d.S + j];
  } else {
    fv = rhs(m, w, y, a.p, lane);
  }
  if (f && lane < N) f[(int64_t)lane * a.ld + c] = fv;
}

template <int NP>
__global__ __launch_bounds__(256) void k_lu_solve(int64_t nmat, int n, const double* A, double* b, int32_t* info) {
  __shared__ int slots[4][64];
  const int wv = threadIdx.x / WAVE;
  const int64_t mi = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
  if (mi >= nmat) return;
  const int lane = lane_id();
  double row[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) row[j] = (lane < n && j < n) ? A[((size_t)mi * n + lane) * n + j] : 0.0;
  int mystep;
  double myrdiag;
  const int rc = lu_factor<NP>(row, n, lane, mystep, myrdiag);
  if (lane == 0) info[mi] = rc;
  if (rc) return;
  const int src = permute_rows<NP>(row, n, lane, mystep, myrdiag, slots[wv]);
  const double bi = lane < n ? b[(size_t)mi * n + lane] : 0.0;
  const double x = lu_solve<NP>(row, n, lane, src, myrdiag, bi);
  if (lane < n) b[(size_t)mi * n + lane] = x;
}

// getrf of each matrix: LU in LAPACK's layout (rows in pivot order) and ipiv.
template <int NP>
__global__ __launch_bounds__(256) void k_lu_factor(int64_t nmat, int n, const double* A, double* LU, int32_t* ipiv,
                                                   int32_t* info) {
  __shared__ int slots[4][64];
  const int wv = threadIdx.x / WAVE;
  const int64_t mi = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
  if (mi >= nmat) return;
  const int lane = lane_id();
  double row[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) row[j] = (lane < n && j < n) ? A[((size_t)mi * n + lane) * n + j] : 0.0;
  int mystep, myipiv = 0;
  double myrdiag;
  const int rc = lu_factor<NP>(row, n, lane, mystep, myrdiag, false, &myipiv);
  if (lane == 0) info[mi] = rc;
  if (rc) return;  // some rows never became pivots: no permutation to apply
  permute_rows<NP>(row, n, lane, mystep, myrdiag, slots[wv]);
  if (lane < n) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (j < n) LU[((size_t)mi * n + lane) * n + j] = row[j];
    ipiv[(size_t)mi * n + lane] = myipiv;
  }
}

// ---------------------------------------------------------------- workgroup path (64 < N <= 256)
// One cell per 256-thread workgroup; each workgroup owns a scratch slot of two
// NP x NP matrices.  The grid is persistent (cells come from the queue).
// The mechanism tables stay in global memory (L2-resident, shared by all
// workgroups) so that two workgroups fit in one CU's LDS.
template <bool PROF>
__global__ __launch_bounds__(WG, 2) void k_integrate_wg(IntArgs a, WgTerms tl, double* scratch, int NP) {
  extern __shared__ __align__(16) uint8_t lds[];
  const MechView m = make_view(a.blob, a);
  const WgWs w = make_wg_ws((double*)lds, a.d.R, NP);
  double* Sx = scratch + (size_t)blockIdx.x * 2 * NP * NP;
  double* Mx = Sx + (size_t)NP * NP;
  for (int i = threadIdx.x; i < NP * NP; i += WG) Sx[i] = 0.0;
  for (int i = threadIdx.x; i < wg_ntb(a.d); i += WG) w.tbd[i] = m.tbd[i];
  __syncthreads();
  if (threadIdx.x == 0) w.flag[3] = atomicAdd(a.queue, 1);
  __syncthreads();
  int64_t idx = w.flag[3];
  __syncthreads();
  const int64_t lim = a.nactive ? (int64_t)*a.nactive : a.ncells;
  while (idx < lim) {
    const int64_t c = a.order ? (int64_t)a.order[idx] : idx;
    wg_integrate_cell<PROF>(m, w, tl, Sx, Mx, NP, a, c);
    if (threadIdx.x == 0) w.flag[3] = atomicAdd(a.queue, 1);
    __syncthreads();
    idx = w.flag[3];
    __syncthreads();
  }
}

// (mechanism tables read from global memory, as in the integrator)
// The same launch structure with the Seulex-family integrator.
template <bool PROF>
__global__ __launch_bounds__(WG, 2) void k_integrate_wg_sx(IntArgs a, WgTerms tl, double* scratch, int NP) {
  extern __shared__ __align__(16) uint8_t lds[];
  const MechView m = make_view(a.blob, a);
  const WgWs w = make_wg_ws((double*)lds, a.d.R, NP);
  double* Sx = scratch + (size_t)blockIdx.x * 2 * NP * NP;
  double* Mx = Sx + (size_t)NP * NP;
  for (int i = threadIdx.x; i < NP * NP; i += WG) Sx[i] = 0.0;
  for (int i = threadIdx.x; i < wg_ntb(a.d); i += WG) w.tbd[i] = m.tbd[i];
  __syncthreads();
  if (threadIdx.x == 0) w.flag[3] = atomicAdd(a.queue, 1);
  __syncthreads();
  int64_t idx = w.flag[3];
  __syncthreads();
  const int64_t lim = a.nactive ? (int64_t)*a.nactive : a.ncells;
  while (idx < lim) {
    const int64_t c = a.order ? (int64_t)a.order[idx] : idx;
    wg_integrate_cell_sx<PROF>(m, w, tl, Sx, Mx, NP, a, c);
    if (threadIdx.x == 0) w.flag[3] = atomicAdd(a.queue, 1);
    __syncthreads();
    idx = w.flag[3];
    __syncthreads();
  }
}

__global__ __launch_bounds__(WG) void k_rhs_jac_wg(IntArgs a, WgTerms tl, double* scratch, int NP, const double* st,
                                                   double* f, double* J) {
  extern __shared__ __align__(16) uint8_t lds[];
  const MechView m = make_view(a.blob, a);
  const WgWs w = make_wg_ws((double*)lds, a.d.R, NP);
  double* Sx = scratch + (size_t)blockIdx.x * NP * NP;
  for (int i = threadIdx.x; i < NP * NP; i += WG) Sx[i] = 0.0;
  for (int i = threadIdx.x; i < wg_ntb(a.d); i += WG) w.tbd[i] = m.tbd[i];
  __syncthreads();
  const int t = threadIdx.x, N = m.d.N;
  for (int64_t c = blockIdx.x; c < a.ncells; c += gridDim.x) {
    const double y = t < N ? st[(int64_t)t * a.ld + c] : 0.0;
    double fv;
    if (J) {
      fv = wg_jac(m, w, tl, Sx, NP, y, a.p);
      for (int idx = t; idx < N * N; idx += WG) {
        const int i = idx / N, j = idx - i * N;
        double v;
        if (i == 0) v = w.jTr[j];
        else if (j == 0) v = w.jT0[i];
        else v = m.iW[j - 1] * (m.W[i - 1] * (Sx[(size_t)i * NP + j] + w.ad[i]) + w.gam[i]);
        J[(size_t)c * N * N + idx] = v;
      }
    } else {
      fv = wg_rhs(m, w, y, a.p);
    }
    if (f && t < N) f[(int64_t)t * a.ld + c] = fv;
    __syncthreads();
  }
}

__global__ __launch_bounds__(WG) void k_lu_wg(int64_t nmat, int n, const double* A, double* b, int32_t* info,
                                              double* scratch, int NP, double* LU, int32_t* ipiv) {
  extern __shared__ __align__(16) uint8_t lds[];
  const WgWs w = make_wg_ws((double*)lds, 0, NP);
  double* Mx = scratch + (size_t)blockIdx.x * NP * NP;
  const int t = threadIdx.x;
  for (int64_t mi = blockIdx.x; mi < nmat; mi += gridDim.x) {
    for (int idx = t; idx < NP * NP; idx += WG) {
      const int i = idx / NP, j = idx - i * NP;
      Mx[idx] = (i < n && j < n) ? A[((size_t)mi * n + i) * n + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    const int rc = wg_lu(w, Mx, NP);
    if (t == 0) info[mi] = rc;
    if (LU) {  // factors only: Mx holds them in LAPACK's layout (rows interchanged)
      for (int idx = t; idx < n * n; idx += WG) LU[(size_t)mi * n * n + idx] = Mx[(size_t)(idx / n) * NP + idx % n];
      if (t < n) ipiv[(size_t)mi * n + t] = w.piv[t];
    } else if (rc == 0) {
      const double x = wg_solve(w, Mx, NP, t < n ? b[(size_t)mi * n + t] : 0.0);
      if (t < n) b[(size_t)mi * n + t] = x;
    }
    __syncthreads();
  }
}

__global__ void k_set_arrhenius(uint8_t* blob, MechDims d, const int32_t* perm, const double* lnA, const double* b,
                                const double* th) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.R) return;
  const int o = perm[r];  // internal index -> descriptor index
  ((double*)(blob + d.o_lnA))[r] = lnA[o];
  ((double*)(blob + d.o_b))[r] = b[o];
  ((double*)(blob + d.o_th))[r] = th[o];
}

// Cost ordering of the work queue: cells are bucketed by floor(log2(previous
// step count + 1)) and the buckets are handed out largest first, so the
// longest cells start early and the tail of the persistent launch stays short.
// The order inside a bucket is arbitrary; results do not depend on it.
constexpr int NBUCKET = 32;

__device__ __forceinline__ int cost_bucket(int32_t s) {
  const unsigned v = (unsigned)min(max(s, 0), (1 << 30)) + 1u;
  return 31 - __clz(v);
}

// A cell enters the queue unless excl[i] >= 0 (a mapped cell); with steps
// NULL every cell falls in one bucket (plain compaction).
__device__ __forceinline__ bool queued(const int32_t* excl, int64_t i) { return !excl || excl[i] < 0; }

__global__ void k_order_count(const int32_t* steps, const int32_t* excl, int64_t n, int* cnt) {
  __shared__ int loc[NBUCKET];
  if (threadIdx.x < NBUCKET) loc[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && queued(excl, i)) atomicAdd(&loc[steps ? cost_bucket(steps[i]) : 0], 1);
  __syncthreads();
  if (threadIdx.x < NBUCKET && loc[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], loc[threadIdx.x]);
}

// cnt[0..31] counts, cnt[32..63] bucket cursors, cnt[64] the queue length
__global__ void k_order_clear(int* cnt) {
  if (threadIdx.x <= 2 * NBUCKET) cnt[threadIdx.x] = 0;
}

__global__ void k_order_scan(int* cnt) {
  if (threadIdx.x == 0) {
    int off = 0;
    for (int b = NBUCKET - 1; b >= 0; --b) {
      cnt[NBUCKET + b] = off;
      off += cnt[b];
    }
    cnt[2 * NBUCKET] = off;
  }
}

__global__ void k_order_scatter(const int32_t* steps, const int32_t* excl, int64_t n, int* cnt, int32_t* order) {
  __shared__ int loc[NBUCKET], base[NBUCKET];
  if (threadIdx.x < NBUCKET) loc[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n && queued(excl, i);
  int b = 0, r = 0;
  if (in) {
    b = steps ? cost_bucket(steps[i]) : 0;
    r = atomicAdd(&loc[b], 1);
  }
  __syncthreads();
  if (threadIdx.x < NBUCKET && loc[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cnt[NBUCKET + threadIdx.x], loc[threadIdx.x]);
  __syncthreads();
  if (in) order[base[b] + r] = (int32_t)i;
}

// ------------------------------------------------ reference-cell mapping (section 2.2)
// Low-reactivity zone: z = z0 + sum_k w_k Y_k <= z_max (species in index
// order, fused multiply-adds).  The reference is the zone cell of lowest
// index; zone cells within dT of its temperature take its increment instead of
// being integrated.  rm[0] holds the reference index (~0 if the zone is
// empty), rm[1..N] the reference's initial state.
__global__ void k_refmap_init(unsigned long long* rm) {
  if (threadIdx.x == 0) rm[0] = ~0ull;
}

__global__ void k_refmap_zone(const double* st, int64_t ld, int64_t n, int K, const double* wt, double z0,
                              double zmax, int32_t* ref_of, unsigned long long* rm) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool zone = false;
  if (c < n) {
    double z = z0;
    for (int k = 0; k < K; ++k) z = __builtin_fma(wt[k], st[(int64_t)(k + 1) * ld + c], z);
    zone = z <= zmax;
    ref_of[c] = zone ? -2 : -1;
  }
  // lanes hold consecutive cells: the lowest zone lane is the wave's candidate
  const unsigned long long mask = __ballot(zone);
  if (mask && lane_id() == __ffsll((long long)mask) - 1) atomicMin(rm, (unsigned long long)c);
}

__global__ void k_refmap_mark(double* st, int64_t ld, int64_t n, int N, double dT, int32_t* ref_of,
                              unsigned long long* rm) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const unsigned long long r = rm[0];
  const bool have = r != ~0ull;
  const bool mapped = have && (unsigned long long)c != r && ref_of[c] == -2 && fabs(st[c] - st[r]) <= dT;
  ref_of[c] = mapped ? (int32_t)r : -1;
  if (have && (unsigned long long)c == r) {
    double* y0 = (double*)(rm + 1);
    for (int i = 0; i < N; ++i) y0[i] = st[(int64_t)i * ld + c];
  }
}

__global__ void k_refmap_apply(double* st, int64_t ld, int64_t n, int N, const int32_t* ref_of,
                               const unsigned long long* rm, double* h, int32_t* steps, int32_t* rejects,
                               int32_t* status, unsigned long long* failed) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int32_t r = ref_of[c];
  if (r < 0) return;
  const double* y0 = (const double*)(rm + 1);
  for (int i = 0; i < N; ++i) {
    const int64_t o = (int64_t)i * ld;
    st[o + c] = st[o + c] + (st[o + r] - y0[i]);
  }
  h[c] = h[r];
  if (steps) steps[c] = 0;
  if (rejects) rejects[c] = 0;
  status[c] = status[r];
  if (failed && status[r] != 0) atomicAdd(failed, 1ull);
}

}  // namespace

// Device scratch of chem_integrate_noalloc: the persistent work cursor, the
// cost-order bucket counters and the cost-ordered queue, for callers that
// cannot allocate.  One copy per GPU, held until the process ends.  Layout:
// [0, 4) cursor; [256, 528) bucket counters; [1024, end) queue (int32).
constexpr size_t NOALLOC_BYTES = (size_t)2 << 20;
constexpr size_t NOALLOC_CNT_OFF = 256, NOALLOC_ORDER_OFF = 1024;
constexpr int64_t NOALLOC_MAX_ORDER = (int64_t)((NOALLOC_BYTES - NOALLOC_ORDER_OFF) / sizeof(int32_t));
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

// ================================================================ host side
namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(CHEM_EHIP, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

struct Variant {
  int persistent = 1, wpb = 4, grid_mult = 1;  // grid_mult: workgroups per CU on the workgroup path
  // Jacobian slots shared by a workgroup's waves: -1 auto (the most waves that
  // fit, when more than with private blocks), 0 none (wpb private blocks),
  // n > 0 n slots for pool_waves waves
  int pool = -1, pool_waves = 0;
  bool grid_mult_set = false;  // grid_mult given by an option or the autotuner (workgroup path)
};

// Device address of `scratch` on the current device, looked up once per
// device.  The array's name is only a host-side stand-in: kernels get this
// address, never the name.
std::mutex g_scr_mu;
std::map<int, uint8_t*> g_scr_addr;

int noalloc_scratch(int dev, uint8_t** out) {
  std::lock_guard<std::mutex> lk(g_scr_mu);
  auto it = g_scr_addr.find(dev);
  if (it == g_scr_addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CHEM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scr_addr.emplace(dev, (uint8_t*)p).first;
  }
  *out = it->second;
  return 0;
}

struct GraphKey {
  std::vector<uintptr_t> v;
  bool operator<(const GraphKey& o) const { return v < o.v; }
};

}  // namespace

struct chem_mech {
  MechDims d{};
  int device = 0, ncu = 0, max_lds = 0;
  uint8_t* blob = nullptr;  // device, LDS-staged part
  double* nasa = nullptr;
  int32_t* perm = nullptr;  // device: internal -> descriptor reaction index
  std::vector<int32_t> h_perm;
  int* queue = nullptr;     // device work cursor
  unsigned long long* failed = nullptr;  // device: cells of the last integration with a nonzero status
  int32_t* st_buf = nullptr;  // library status array when the caller passes none (reference mapping)
  uint8_t* noalloc_scr = nullptr;  // this device's copy of `scratch` (device address)
  int64_t st_cap = 0;
  int32_t* order = nullptr; // device cost order of the queue
  int64_t order_cap = 0;
  int* order_cnt = nullptr; // device bucket counters and cursors [64], queue length [1]
  // reference-cell mapping: reference index + its initial state, zone flags
  unsigned long long* rm_buf = nullptr;
  int32_t* rm_flags = nullptr;
  int64_t rm_cap = 0;
  Variant tuned;
  bool has_tuned = false;
  // cached graph of the persistent launch
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
  GraphKey gkey;
  // adjoint workspace and incidence lists
  void* adj_ws = nullptr;
  size_t adj_ws_bytes = 0;
  int32_t* adj_sptr = nullptr;
  uint32_t* adj_sent = nullptr;
  int32_t* adj_tptr = nullptr;
  uint32_t* jsched = nullptr;  // balanced species-scatter schedule of the Jacobian (wavefront path)
  int jsched_it = 0;
  uint32_t* adj_tent = nullptr;
  uint32_t* adj_chunk = nullptr;  // wavefront path: the sent lists cut into <= 64 chunks, [cw][64]
  int32_t* adj_cspan = nullptr;   // [K] first chunk | count << 8
  int adj_cw = 0;
  // workgroup path (64 < N <= 256): Jacobian term lists and per-workgroup scratch
  bool wg = false;
  int wg_np = 0;             // N rounded up to a multiple of 16
  int32_t* wg_gptr = nullptr;
  uint32_t* wg_grp = nullptr;
  uint64_t* wg_term = nullptr;
  int32_t* wg_seg = nullptr;  // [WG][4] term segment per thread (first, end, row, partner)
  double* wg_scr = nullptr;
  size_t wg_scr_bytes = 0;
};

namespace {

int np_for(int N) {
  if (N <= 16) return 16;
  if (N <= 32) return 32;
  if (N <= 56) return 56;
  if (N <= 64) return 64;
  return 0;
}

size_t cell_bytes(const MechDims& d) { return (size_t)cell_ws_doubles(d.N, d.S, d.R, d.R0) * sizeof(double); }

int max_wpb(const chem_mech* m) {
  const size_t avail = (size_t)m->max_lds - m->d.lds_bytes;
  int w = (int)(avail / cell_bytes(m->d));
  return std::min(w, np_for(m->d.N) <= 16 ? MAX_WPB : 4);
}

IntArgs base_args(const chem_mech* m) {
  IntArgs a{};
  a.blob = m->blob;
  a.nasa = m->nasa;
  a.jsched = m->jsched;
  a.jsched_it = m->jsched_it;
  a.d = m->d;
  a.cell_doubles = cell_ws_doubles(m->d.N, m->d.S, m->d.R, m->d.R0);
  return a;
}

template <class F>
int with_np(int N, F&& f) {
  switch (np_for(N)) {
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 56: return f(std::integral_constant<int, 56>());
    case 64: return f(std::integral_constant<int, 64>());
  }
  return fail(CHEM_EUNSUPPORTED, "state size N = " + std::to_string(N) + " exceeds the compiled limit 64");
}

template <int NP>
int set_lds_limit(const void* fn, size_t bytes) {
  HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return 0;
}

// LDS of the workgroup-path kernels (workspace only: they read the
// mechanism tables from global memory)
size_t wg_lds_bytes(const chem_mech* m) {
  return (size_t)wg_ws_doubles(m->d.R, m->wg_np, wg_ntb(m->d)) * sizeof(double);
}

WgTerms wg_terms(const chem_mech* m) {
  WgTerms t;
  t.gptr = m->wg_gptr;
  t.grp = m->wg_grp;
  t.term = m->wg_term;
  t.seg = m->wg_seg;
  return t;
}

// Persistent grid of the workgroup path: one workgroup per CU and LDS slot.
int wg_grid(const chem_mech* m, int64_t items, int per_cu_cap = 0) {
  int per_cu = std::max(1, (int)(m->max_lds / wg_lds_bytes(m)));
  if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)m->ncu * per_cu, items));
}

// Scratch for `slots` workgroups of `mats` NP x NP matrices each (grown lazily;
// never called during graph capture).
int ensure_wg_scratch(chem_mech* m, int slots, int mats) {
  const size_t need = (size_t)slots * mats * m->wg_np * m->wg_np * sizeof(double);
  if (m->wg_scr_bytes >= need) return 0;
  hipFree(m->wg_scr);
  m->wg_scr = nullptr;
  m->wg_scr_bytes = 0;
  if (hipMalloc(&m->wg_scr, need) != hipSuccess) return fail(CHEM_ENOMEM, "workgroup scratch allocation failed");
  m->wg_scr_bytes = need;
  return 0;
}

int launch_integrate_wg(chem_mech* m, const IntArgs& a0, hipStream_t s, int per_cu = 0) {
  IntArgs a = a0;
  const int grid = wg_grid(m, a.ncells, per_cu);
  if ((size_t)grid * 2 * m->wg_np * m->wg_np * sizeof(double) > m->wg_scr_bytes)
    return fail(CHEM_EINVAL, "workgroup scratch not prepared");
  const size_t lds = wg_lds_bytes(m);
  auto kern = a.method == 2 ? (a.prof ? k_integrate_wg_sx<true> : k_integrate_wg_sx<false>)
                            : (a.prof ? k_integrate_wg<true> : k_integrate_wg<false>);
  HIPCHK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  a.queue = m->queue;
  a.failed = m->failed;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, m->queue, m->failed);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), lds, s, a, wg_terms(m), m->wg_scr, m->wg_np);
  HIPCHK(hipGetLastError());
  return 0;
}

int launch_rhs_jac_wg(chem_mech* m, const IntArgs& a, const double* st, double* f, double* J, hipStream_t s) {
  const int grid = wg_grid(m, a.ncells);
  const int rc = ensure_wg_scratch(m, grid, 2);
  if (rc) return rc;
  const size_t lds = wg_lds_bytes(m);
  HIPCHK(hipFuncSetAttribute((const void*)k_rhs_jac_wg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_rhs_jac_wg, dim3(grid), dim3(WG), lds, s, a, wg_terms(m), m->wg_scr, m->wg_np, st, f, J);
  HIPCHK(hipGetLastError());
  return 0;
}

// Shared-slot layout of the Rosenbrock kernel: waves per workgroup and
// slots.  The most waves (up to 8) for which three slots fit (two below six
// waves); {0, 0} when no layout beats the private-Jacobian one (N <= 16, or
// the Seulex integrator, whose steps reuse one Jacobian for many matrices).
struct PoolLayout {
  int waves = 0, slots = 0;
  size_t lds = 0;
};
size_t pool_lds(const chem_mech* m, int waves, int slots) {
  const MechDims& d = m->d;
  return (size_t)d.lds_bytes + (size_t)waves * wave_rates_doubles(d.R, d.R0) * sizeof(double) + 64 +
         (size_t)slots * d.N * d.S * sizeof(double);
}
PoolLayout pool_layout(const chem_mech* m, int method, int want_waves = 0, int want_slots = 0) {
  PoolLayout L;
  if (m->wg || method == 2 || np_for(m->d.N) <= 16) return L;
  for (int w = 8; w > max_wpb(m); --w) {
    if (want_waves > 0 && w != want_waves) continue;
    const int s = want_slots > 0 ? std::min(want_slots, w) : (w >= 6 ? 3 : 2);
    if (pool_lds(m, w, s) <= (size_t)m->max_lds) {
      L.waves = w;
      L.slots = s;
      L.lds = pool_lds(m, w, s);
      return L;
    }
  }
  return L;
}

int launch_integrate_pool(chem_mech* m, const IntArgs& a0, const Variant& v, const PoolLayout& L, hipStream_t s,
                         int* queue) {
  IntArgs a = a0;
  a.cell_doubles = wave_rates_doubles(m->d.R, m->d.R0);
  a.pool_slots = L.slots;
  return with_np(m->d.N, [&](auto npc) -> int {
    constexpr int NP = decltype(npc)::value;
    auto kern = (a.prof || a.jac_fd || a.lu_nopiv) ? k_integrate_pool<NP, true> : k_integrate_pool<NP, false>;
    if (set_lds_limit<NP>((const void*)kern, L.lds)) return CHEM_EHIP;
    int grid;
    if (v.persistent) {
      int occ = 0;
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, L.waves * WAVE, L.lds));
      occ = std::max(occ, 1);
      const int64_t need = (a.ncells + L.waves - 1) / L.waves;
      grid = (int)std::min<int64_t>((int64_t)m->ncu * occ * std::max(1, v.grid_mult), need);
      a.queue = queue;
    } else {
      a.queue = nullptr;
      grid = (int)((a.ncells + L.waves - 1) / L.waves);
    }
    a.failed = m->failed;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, a.queue, m->failed);
    HIPCHK(hipGetLastError());
    if (grid > 0) {
      hipLaunchKernelGGL(kern, dim3(grid), dim3(L.waves * WAVE), L.lds, s, a);
      HIPCHK(hipGetLastError());
    }
    return 0;
  });
}

// queue: the persistent work cursor (the mechanism's own, or the no-allocation
// entry point's device scratch)
int launch_integrate(chem_mech* m, const IntArgs& a0, const Variant& v, hipStream_t s, int* queue = nullptr) {
  if (!queue) queue = m->queue;
  if (m->wg) return launch_integrate_wg(m, a0, s, v.grid_mult_set ? v.grid_mult : 0);
  if (v.pool != 0) {
    const PoolLayout L = pool_layout(m, a0.method, v.pool_waves, v.pool > 0 ? v.pool : 0);
    if (L.waves > 0) return launch_integrate_pool(m, a0, v, L, s, queue);
  }
  IntArgs a = a0;
  const int wpb = std::max(1, std::min(v.wpb, max_wpb(m)));
  if (wpb < 1) return fail(CHEM_EUNSUPPORTED, "mechanism workspace does not fit in LDS");
  const size_t lds = m->d.lds_bytes + (size_t)wpb * cell_bytes(m->d);
  return with_np(m->d.N, [&](auto npc) -> int {
    constexpr int NP = decltype(npc)::value;
    // the instrumented kernel also carries the ablation switches
    auto kern = a.method == 2 ? (a.prof ? k_integrate_sx<NP, true> : k_integrate_sx<NP, false>)
                : (a.prof || a.jac_fd || a.lu_nopiv) ? k_integrate<NP, true> : k_integrate<NP, false>;
    const void* fn = (const void*)kern;
    if (set_lds_limit<NP>(fn, lds)) return CHEM_EHIP;
    int grid;
    if (v.persistent) {
      int occ = 0;
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, wpb * WAVE, lds));
      occ = std::max(occ, 1);
      const int64_t need = (a.ncells + wpb - 1) / wpb;
      grid = (int)std::min<int64_t>((int64_t)m->ncu * occ * std::max(1, v.grid_mult), need);
      a.queue = queue;
    } else {
      a.queue = nullptr;
      grid = (int)((a.ncells + wpb - 1) / wpb);
    }
    a.failed = m->failed;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, a.queue, m->failed);
    HIPCHK(hipGetLastError());
    if (grid > 0) {
      hipLaunchKernelGGL(kern, dim3(grid), dim3(wpb * WAVE), lds, s, a);
      HIPCHK(hipGetLastError());
    }
    return 0;
  });
}

// Builds the queue in m->order: cells with excl[i] >= 0 left out (if excl is
// given), the rest by descending cost bucket of steps (if given); the queue
// length goes to m->order_cnt[2 NBUCKET].
int launch_order(chem_mech* m, const int32_t* steps, const int32_t* excl, int64_t ncells, hipStream_t s,
                 int32_t* order = nullptr, int* cnt = nullptr) {
  if (!order) order = m->order;
  if (!cnt) cnt = m->order_cnt;
  const int nb = (int)((ncells + 255) / 256);
  hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(128), 0, s, cnt);
  hipLaunchKernelGGL(k_order_count, dim3(nb), dim3(256), 0, s, steps, excl, ncells, cnt);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, cnt);
  hipLaunchKernelGGL(k_order_scatter, dim3(nb), dim3(256), 0, s, steps, excl, ncells, cnt, order);
  HIPCHK(hipGetLastError());
  return 0;
}

// Zone test, reference choice and marking of the mapped cells (before the
// integration), and the increments of the mapped cells (after it).
int launch_refmap_mark(chem_mech* m, const chem_refmap& rm, int32_t* ref_of, double* state, int64_t ld,
                       int64_t ncells, hipStream_t s) {
  const int nb = (int)((ncells + 255) / 256);
  hipLaunchKernelGGL(k_refmap_init, dim3(1), dim3(64), 0, s, m->rm_buf);
  hipLaunchKernelGGL(k_refmap_zone, dim3(nb), dim3(256), 0, s, state, ld, ncells, m->d.K, rm.weight, rm.z0,
                     rm.z_max, ref_of, m->rm_buf);
  hipLaunchKernelGGL(k_refmap_mark, dim3(nb), dim3(256), 0, s, state, ld, ncells, m->d.N, rm.dT, ref_of, m->rm_buf);
  HIPCHK(hipGetLastError());
  return 0;
}

int launch_refmap_apply(chem_mech* m, const int32_t* ref_of, double* state, int64_t ld, int64_t ncells, double* h,
                        int32_t* steps, int32_t* rejects, int32_t* status, hipStream_t s) {
  const int nb = (int)((ncells + 255) / 256);
  hipLaunchKernelGGL(k_refmap_apply, dim3(nb), dim3(256), 0, s, state, ld, ncells, m->d.N, ref_of, m->rm_buf, h,
                     steps, rejects, status, m->failed);
  HIPCHK(hipGetLastError());
  return 0;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* chem_last_error(void) { return g_err.c_str(); }

int chem_max_n(void) { return 255; }

int chem_load_mechanism(const chem_mech_desc* desc, chem_mech** out) {
  if (!desc || !out) return fail(CHEM_EINVAL, "null descriptor or output pointer");
  *out = nullptr;
  const int K = desc->n_species, R = desc->n_reactions;
  if (K < 1 || R < 0) return fail(CHEM_EINVAL, "need n_species >= 1 and n_reactions >= 0");
  if (K > 254) return fail(CHEM_EUNSUPPORTED, "more than 254 species");
  if (!desc->W || !desc->nasa7 || (R > 0 && (!desc->rtype || !desc->reac || !desc->prod || !desc->lnA ||
                                             !desc->b || !desc->theta)))
    return fail(CHEM_EINVAL, "missing mechanism array");
  const int N = K + 1;
  const bool wg = np_for(N) == 0;  // N > 64: one cell per workgroup
  if (wg && R >= 65536) return fail(CHEM_EUNSUPPORTED, "more than 65535 reactions for N > 64");
  for (int k = 0; k < K; ++k)
    if (!(desc->W[k] > 0.0) || !std::isfinite(desc->W[k])) return fail(CHEM_EINVAL, "molar masses must be positive");
  if (!finite_all(desc->nasa7, (size_t)15 * K)) return fail(CHEM_EINVAL, "non-finite NASA-7 coefficient");
  for (int k = 0; k < K; ++k) {
    const double* row = desc->nasa7 + 15 * k;
    for (int i = 0; i <= 100; ++i) {
      const double T = 200.0 + 58.0 * i;
      const double* a = T > row[0] ? row + 8 : row + 1;
      const double cp = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
      if (!(cp > 0.0)) return fail(CHEM_EINVAL, "cp <= 0 on [200, 6000] K for species " + std::to_string(k));
    }
  }
  // reaction order: elementary, third-body, Troe (stable within each type)
  std::vector<int> order;
  for (int t = 0; t < 3; ++t)
    for (int r = 0; r < R; ++r) {
      const int ty = desc->rtype[r];
      if (ty < 0 || ty > 2) return fail(CHEM_EINVAL, "reaction type must be 0, 1 or 2");
      if (ty == t) order.push_back(r);
    }
  int R0 = 0, R1 = 0;
  for (int r = 0; r < R; ++r) {
    if (desc->rtype[r] == 0) ++R0;
    if (desc->rtype[r] <= 1) ++R1;
  }
  if (desc->n_elements < 0 || (desc->n_elements > 0 && !desc->elem))
    return fail(CHEM_EINVAL, "n_elements must be >= 0, with an elem array when > 0");
  if (desc->n_elements > 0) {
    // every reaction conserves each element (a third body is not a species)
    const int E = desc->n_elements;
    for (int r = 0; r < R; ++r) {
      for (int e = 0; e < E; ++e) {
        long long bal = 0;
        for (int s2 = 0; s2 < 3; ++s2) {
          const int a = desc->reac[3 * r + s2], b = desc->prod[3 * r + s2];
          if (a < -1 || a >= K || b < -1 || b >= K)
            return fail(CHEM_EINVAL, "species index out of range in reaction " + std::to_string(r));
          if (a >= 0) bal -= desc->elem[(size_t)a * E + e];
          if (b >= 0) bal += desc->elem[(size_t)b * E + e];
        }
        if (bal != 0)
          return fail(CHEM_EINVAL, "reaction " + std::to_string(r) + " does not conserve element " + std::to_string(e));
      }
    }
  }
  if (R > R0 && !desc->eff) return fail(CHEM_EINVAL, "third-body reactions need efficiencies");
  if (R > R1 && (!desc->troe || !desc->low)) return fail(CHEM_EINVAL, "Troe reactions need troe and low data");

  MechDims d{};
  d.K = K;
  d.R = R;
  d.N = N;
  d.S = wg ? N + 1 : np_for(N) + 1;  // odd (NP is a multiple of 8), with padding columns after N
  d.R0 = R0;
  d.R1 = R1;
  // species -> (reaction, net nu) incidence, ascending internal reaction index
  std::vector<std::vector<uint32_t>> inc(K);
  std::vector<uint64_t> sp(R);
  for (int ri = 0; ri < R; ++ri) {
    const int r = order[ri];
    int cnt[2] = {0, 0};
    int slots[2][3] = {{K, K, K}, {K, K, K}};
    std::map<int, int> nu;
    for (int side = 0; side < 2; ++side) {
      const int32_t* arr = (side == 0 ? desc->reac : desc->prod) + 3 * r;
      for (int s = 0; s < 3; ++s) {
        const int v = arr[s];
        if (v < -1 || v >= K) return fail(CHEM_EINVAL, "species index out of range in reaction " + std::to_string(r));
        if (v < 0) continue;
        slots[side][cnt[side]++] = v;
        nu[v] += side == 0 ? -1 : 1;
      }
    }
    uint64_t w = 0;
    for (int s = 0; s < 3; ++s) w |= (uint64_t)slots[0][s] << (8 * s);
    for (int s = 0; s < 3; ++s) w |= (uint64_t)slots[1][s] << (8 * (s + 3));
    w |= (uint64_t)cnt[0] << 48;
    w |= (uint64_t)cnt[1] << 56;
    sp[ri] = w;
    for (auto& kv : nu)
      if (kv.second != 0) inc[kv.first].push_back(((uint32_t)ri << 8) | (uint8_t)(int8_t)kv.second);
  }
  std::vector<int32_t> cptr(K + 1, 0);
  std::vector<uint32_t> cent;
  for (int k = 0; k < K; ++k) {
    cptr[k] = (int32_t)cent.size();
    cent.insert(cent.end(), inc[k].begin(), inc[k].end());
  }
  cptr[K] = (int32_t)cent.size();
  d.L = (int)cent.size();
  // Schedule of the Jacobian's species scatter on the wavefront path: the
  // incidence entries dealt over species in rounds (one entry of every species
  // that has one left per round), cut into iterations of 64 lanes; entry
  // (r << 16) | (k << 8) | (uint8)nu, ~0u for an idle lane.  Every lane then
  // processes about L / 64 entries instead of its own species' list.
  std::vector<uint32_t> jsched;
  if (!wg) {
    if (R > 65535) return fail(CHEM_EUNSUPPORTED, "more than 65535 reactions for N <= 64");
    std::vector<uint32_t> seq;
    for (size_t t = 0;; ++t) {
      bool any = false;
      for (int k = 0; k < K; ++k) {
        if (t >= inc[k].size()) continue;
        const uint32_t e = inc[k][t];
        seq.push_back(((e >> 8) << 16) | ((uint32_t)k << 8) | (e & 0xFF));
        any = true;
      }
      if (!any) break;
    }
    const size_t nit = (seq.size() + 63) / 64;
    jsched.assign(std::max<size_t>(nit, 1) * 64, ~0u);
    std::copy(seq.begin(), seq.end(), jsched.begin());
  }
  // third-body lists (non-unit efficiencies) and Troe data, internal order
  std::vector<int32_t> tbp(R - R0 + 1, 0), tbs;
  std::vector<double> tbd;
  for (int ri = R0; ri < R; ++ri) {
    const int r = order[ri];
    int n = 0;
    for (int k = 0; k < K; ++k) {
      const double ev = desc->eff[(size_t)r * K + k];
      if (!std::isfinite(ev)) return fail(CHEM_EINVAL, "non-finite efficiency");
      if (ev != 1.0) {
        if (++n > MAXTB) return fail(CHEM_EUNSUPPORTED, "more than 8 non-unit efficiencies in a reaction");
        tbs.push_back(k);
        tbd.push_back(ev - 1.0);
      }
    }
    tbp[ri - R0 + 1] = (int32_t)tbs.size();
  }
  std::vector<double> troe((size_t)TROE_STRIDE * (R - R1), 0.0);
  for (int ri = R1; ri < R; ++ri) {
    const int r = order[ri];
    const double* t = desc->troe + 4 * r;
    const double* lo = desc->low + 3 * r;
    if (!(t[1] > 0.0) || !(t[2] > 0.0) || !finite_all(t, 4) || !finite_all(lo, 3))
      return fail(CHEM_EINVAL, "Troe parameters need positive T*** and T*");
    double* o = &troe[(size_t)TROE_STRIDE * (ri - R1)];
    o[0] = t[0];
    o[1] = 1.0 / t[1];
    o[2] = 1.0 / t[2];
    o[3] = t[3];
    o[4] = lo[0];
    o[5] = lo[1];
    o[6] = lo[2];
  }
  // LDS blob layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 15) & ~(size_t)15;
    return (int)o;
  };
  d.o_lnA = take(8 * (size_t)R);
  d.o_b = take(8 * (size_t)R);
  d.o_th = take(8 * (size_t)R);
  d.o_sp = take(8 * (size_t)R);
  d.o_W = take(8 * (size_t)K);
  d.o_iW = take(8 * (size_t)K);
  d.o_cptr = take(4 * (size_t)(K + 1));
  d.o_cent = take(4 * (size_t)std::max(d.L, 1));
  d.o_tbp = take(4 * tbp.size());
  d.o_tbs = take(4 * std::max<size_t>(tbs.size(), 1));
  d.o_tbd = take(8 * std::max<size_t>(tbd.size(), 1));
  d.o_troe = take(8 * std::max<size_t>(troe.size(), 1));  // right after tbd: wg_ntb counts tbd from the gap
  d.lds_bytes = (int)off;
  std::vector<uint8_t> blob(off, 0);
  for (int ri = 0; ri < R; ++ri) {
    const int r = order[ri];
    ((double*)(blob.data() + d.o_lnA))[ri] = desc->lnA[r];
    ((double*)(blob.data() + d.o_b))[ri] = desc->b[r];
    ((double*)(blob.data() + d.o_th))[ri] = desc->theta[r];
    ((uint64_t*)(blob.data() + d.o_sp))[ri] = sp[ri];
  }
  if (!finite_all(desc->lnA, R) || !finite_all(desc->b, R) || !finite_all(desc->theta, R))
    return fail(CHEM_EINVAL, "non-finite Arrhenius parameter");
  for (int k = 0; k < K; ++k) {
    ((double*)(blob.data() + d.o_W))[k] = desc->W[k];
    ((double*)(blob.data() + d.o_iW))[k] = 1.0 / desc->W[k];
  }
  std::memcpy(blob.data() + d.o_cptr, cptr.data(), 4 * cptr.size());
  if (!cent.empty()) std::memcpy(blob.data() + d.o_cent, cent.data(), 4 * cent.size());
  std::memcpy(blob.data() + d.o_tbp, tbp.data(), 4 * tbp.size());
  if (!tbs.empty()) std::memcpy(blob.data() + d.o_tbs, tbs.data(), 4 * tbs.size());
  if (!tbd.empty()) std::memcpy(blob.data() + d.o_tbd, tbd.data(), 8 * tbd.size());
  if (!troe.empty()) std::memcpy(blob.data() + d.o_troe, troe.data(), 8 * troe.size());
  std::vector<double> nasa((size_t)16 * K, 0.0);
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < 15; ++i) nasa[16 * k + i] = desc->nasa7[15 * k + i];
  // adjoint incidence: species -> (reaction, molecule slot) and -> (reaction, efficiency entry)
  std::vector<std::vector<uint32_t>> sinc(K), tinc(K);
  for (int ri = 0; ri < R; ++ri)
    for (int sl = 0; sl < 6; ++sl) {
      const int spc = (int)((sp[ri] >> (8 * sl)) & 0xFF);
      if (spc < K) sinc[spc].push_back(((uint32_t)ri << 3) | (uint32_t)sl);
    }
  if (tbs.size() >= 4096 || R >= (1 << 20)) return fail(CHEM_EUNSUPPORTED, "mechanism too large for the adjoint tables");
  for (int ri = R0; ri < R; ++ri)
    for (int e = tbp[ri - R0]; e < tbp[ri - R0 + 1]; ++e) tinc[tbs[e]].push_back(((uint32_t)ri << 12) | (uint32_t)e);
  std::vector<int32_t> sptr(K + 1, 0), tptr(K + 1, 0);
  std::vector<uint32_t> sent, tent;
  for (int k = 0; k < K; ++k) {
    sptr[k] = (int32_t)sent.size();
    sent.insert(sent.end(), sinc[k].begin(), sinc[k].end());
    tptr[k] = (int32_t)tent.size();
    tent.insert(tent.end(), tinc[k].begin(), tinc[k].end());
  }
  sptr[K] = (int32_t)sent.size();
  tptr[K] = (int32_t)tent.size();
  // the sent lists cut into at most 64 chunks of at most cw entries, a
  // species' chunks consecutive, cw the smallest width that needs <= 64
  // chunks; chunk j is summed by lane j of the adjoint's gather
  std::vector<uint32_t> chunk;
  std::vector<int32_t> cspan(std::max(K, 1), 0);
  int cw = 0;
  if (!wg && K > 0) {
    size_t mx = 0;
    for (int k = 0; k < K; ++k) mx = std::max(mx, sinc[k].size());
    cw = (int)std::max<size_t>(mx, 1);
    for (int w = 1; w <= (int)std::max<size_t>(mx, 1); ++w) {
      size_t nch = 0;
      for (int k = 0; k < K; ++k) nch += std::max<size_t>((sinc[k].size() + w - 1) / w, 1);
      if (nch <= 64) {
        cw = w;
        break;
      }
    }
    cw = (cw + 3) / 4 * 4;
    chunk.assign((size_t)cw * 64, ~0u);
    int j = 0;
    for (int k = 0; k < K; ++k) {
      const int n = (int)sinc[k].size(), nc = std::max((n + cw - 1) / cw, 1);
      cspan[k] = j | (nc << 8);
      for (int q = 0; q < nc; ++q, ++j)
        for (int i = 0; i < cw && q * cw + i < n; ++i) chunk[(size_t)i * 64 + j] = sinc[k][q * cw + i];
    }
    if (j > 64) return fail(CHEM_EUNSUPPORTED, "adjoint gather schedule needs more than 64 chunks");
  }
  if (sent.empty()) sent.push_back(0);
  if (tent.empty()) tent.push_back(0);
  // workgroup-path Jacobian terms: per species row, groups by column, terms in a fixed order
  std::vector<int32_t> wgptr;
  std::vector<uint32_t> wgrp;
  std::vector<uint64_t> wterm;
  std::vector<int32_t> wseg;
  if (wg) {
    wgptr.assign(K + 1, 0);
    for (int k = 0; k < K; ++k) {
      wgptr[k] = (int32_t)wgrp.size();
      std::vector<std::vector<uint64_t>> bycol(K);
      for (int e = cptr[k]; e < cptr[k + 1]; ++e) {
        const int ri = (int)(cent[e] >> 8);
        const uint64_t nu8 = (uint64_t)(uint8_t)(cent[e] & 0xFF);
        uint64_t sl[6];
        for (int q = 0; q < 6; ++q) sl[q] = (sp[ri] >> (8 * q)) & 0xFF;
        for (int q = 0; q < 6; ++q) {
          if ((int)sl[q] >= K) continue;
          const int b0 = q < 3 ? 0 : 3;
          const int qa = b0 + (q - b0 == 0 ? 1 : 0), qb = b0 + (q - b0 == 2 ? 1 : 2);
          bycol[sl[q]].push_back((uint64_t)ri | ((uint64_t)q << 16) | (nu8 << 24) | (sl[qa] << 32) | (sl[qb] << 40));
        }
        if (ri >= R0)
          for (int te = tbp[ri - R0]; te < tbp[ri - R0 + 1]; ++te)
            bycol[tbs[te]].push_back((uint64_t)ri | (6ull << 16) | (nu8 << 24) | ((uint64_t)te << 48));
      }
      for (int l = 0; l < K; ++l) {
        if (bycol[l].empty()) continue;
        wgrp.push_back(((uint32_t)wterm.size() << 8) | (uint32_t)l);
        bycol[l].back() |= (1ull << 19) | ((uint64_t)(l & 0xF) << 20) | ((uint64_t)(l >> 4) << 60);
        wterm.insert(wterm.end(), bycol[l].begin(), bycol[l].end());
      }
    }
    wgptr[K] = (int32_t)wgrp.size();
    wgrp.push_back((uint32_t)wterm.size() << 8);
    if (wterm.size() >= (1u << 24)) return fail(CHEM_EUNSUPPORTED, "too many Jacobian terms");
    if (wterm.empty()) wterm.push_back(0);
    // term segments: thread 1 + k sums row k; the threads that own no row
    // (0 and K+1 ..) take the second half of the longest rows, split at the
    // column group that best balances the two halves
    wseg.assign(4 * WG, -1);
    auto gstart = [&](int g) { return (int32_t)(wgrp[g] >> 8); };
    std::vector<int> byLen(K);
    for (int k = 0; k < K; ++k) {
      byLen[k] = k;
      int32_t* q = &wseg[4 * (1 + k)];
      q[0] = gstart(wgptr[k]);
      q[1] = gstart(wgptr[k + 1]);
      q[2] = k;
    }
    std::stable_sort(byLen.begin(), byLen.end(), [&](int x, int y) {
      return gstart(wgptr[x + 1]) - gstart(wgptr[x]) > gstart(wgptr[y + 1]) - gstart(wgptr[y]);
    });
    int next = 0;
    for (int sp = 0; sp < WG; ++sp) {
      if (sp >= 1 && sp <= K) continue;
      if (next >= K) break;
      const int k = byLen[next++];
      const int32_t tb = gstart(wgptr[k]), te = gstart(wgptr[k + 1]);
      int best = -1;
      int32_t bestw = te - tb;
      for (int g = wgptr[k] + 1; g < wgptr[k + 1]; ++g) {
        const int32_t wmax = std::max(gstart(g) - tb, te - gstart(g));
        if (wmax < bestw) {
          bestw = wmax;
          best = g;
        }
      }
      if (best < 0) continue;  // a single column group stays whole
      int32_t* q = &wseg[4 * (1 + k)];
      q[1] = gstart(best);
      q[3] = sp;
      int32_t* r = &wseg[4 * sp];
      r[0] = gstart(best);
      r[1] = te;
      r[2] = k;
      r[3] = -1;
    }
  }
  chem_mech* m = new chem_mech();
  m->d = d;
  m->wg = wg;
  m->wg_np = wg ? ((N + 15) / 16) * 16 : 0;
  m->h_perm.assign(order.begin(), order.end());
  auto cleanup = [&](int code, const std::string& msg) {
    chem_free_mechanism(m);
    return fail(code, msg);
  };
  if (hipGetDevice(&m->device) != hipSuccess) return cleanup(CHEM_EHIP, "hipGetDevice failed");
  if (noalloc_scratch(m->device, &m->noalloc_scr)) return cleanup(CHEM_EHIP, g_err);
  hipDeviceGetAttribute(&m->ncu, hipDeviceAttributeMultiprocessorCount, m->device);
  hipDeviceGetAttribute(&m->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
  if (!wg && m->max_lds < d.lds_bytes + (int)cell_bytes(d))
    return cleanup(CHEM_EUNSUPPORTED, "mechanism workspace needs more LDS than one workgroup has");
  if (wg && (size_t)m->max_lds < wg_lds_bytes(m))
    return cleanup(CHEM_EUNSUPPORTED, "the workgroup workspace needs more LDS than a workgroup has");
  if (wg) {
    if (hipMalloc(&m->wg_gptr, 4 * wgptr.size()) != hipSuccess || hipMalloc(&m->wg_grp, 4 * wgrp.size()) != hipSuccess ||
        hipMalloc(&m->wg_term, 8 * wterm.size()) != hipSuccess || hipMalloc(&m->wg_seg, 4 * wseg.size()) != hipSuccess)
      return cleanup(CHEM_ENOMEM, "device allocation failed");
    if (hipMemcpy(m->wg_gptr, wgptr.data(), 4 * wgptr.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->wg_grp, wgrp.data(), 4 * wgrp.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->wg_term, wterm.data(), 8 * wterm.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->wg_seg, wseg.data(), 4 * wseg.size(), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(CHEM_EHIP, "upload failed");
  }
  if (hipMalloc(&m->blob, blob.size()) != hipSuccess || hipMalloc(&m->nasa, 8 * nasa.size()) != hipSuccess ||
      hipMalloc(&m->perm, 4 * (size_t)std::max(R, 1)) != hipSuccess || hipMalloc(&m->queue, 64) != hipSuccess ||
      hipMalloc(&m->adj_sptr, 4 * sptr.size()) != hipSuccess || hipMalloc(&m->adj_sent, 4 * sent.size()) != hipSuccess ||
      hipMalloc(&m->adj_tptr, 4 * tptr.size()) != hipSuccess || hipMalloc(&m->adj_tent, 4 * tent.size()) != hipSuccess)
    return cleanup(CHEM_ENOMEM, "device allocation failed");
  if (!chunk.empty()) {
    m->adj_cw = cw;
    if (hipMalloc(&m->adj_chunk, 4 * chunk.size()) != hipSuccess || hipMalloc(&m->adj_cspan, 4 * cspan.size()) != hipSuccess)
      return cleanup(CHEM_ENOMEM, "device allocation failed");
    if (hipMemcpy(m->adj_chunk, chunk.data(), 4 * chunk.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->adj_cspan, cspan.data(), 4 * cspan.size(), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(CHEM_EHIP, "upload failed");
  }
  if (!jsched.empty()) {
    m->jsched_it = (int)(jsched.size() / 64);
    if (hipMalloc(&m->jsched, 4 * jsched.size()) != hipSuccess) return cleanup(CHEM_ENOMEM, "device allocation failed");
    if (hipMemcpy(m->jsched, jsched.data(), 4 * jsched.size(), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(CHEM_EHIP, "upload failed");
  }
  if (hipMemcpy(m->adj_sptr, sptr.data(), 4 * sptr.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->adj_sent, sent.data(), 4 * sent.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->adj_tptr, tptr.data(), 4 * tptr.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->adj_tent, tent.data(), 4 * tent.size(), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(CHEM_EHIP, "upload failed");
  if (hipMemcpy(m->blob, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->nasa, nasa.data(), 8 * nasa.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (R > 0 && hipMemcpy(m->perm, order.data(), 4 * (size_t)R, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemset(m->queue, 0, 64) != hipSuccess)
    return cleanup(CHEM_EHIP, "upload failed");
  // the failed-cell counter shares the 64-byte queue allocation (the cursor is its first word)
  m->failed = reinterpret_cast<unsigned long long*>(reinterpret_cast<uint8_t*>(m->queue) + 8);
  *out = m;
  return CHEM_OK;
}

void chem_free_mechanism(chem_mech* m) {
  if (!m) return;
  if (m->gexec) hipGraphExecDestroy(m->gexec);
  if (m->graph) hipGraphDestroy(m->graph);
  if (m->cap_stream) hipStreamDestroy(m->cap_stream);
  hipFree(m->blob);
  hipFree(m->nasa);
  hipFree(m->perm);
  hipFree(m->queue);
  hipFree(m->adj_ws);
  hipFree(m->order);
  hipFree(m->order_cnt);
  hipFree(m->rm_buf);
  hipFree(m->rm_flags);
  hipFree(m->st_buf);
  hipFree(m->wg_gptr);
  hipFree(m->wg_grp);
  hipFree(m->wg_term);
  hipFree(m->wg_seg);
  hipFree(m->wg_scr);
  hipFree(m->adj_sptr);
  hipFree(m->adj_sent);
  hipFree(m->adj_tptr);
  hipFree(m->adj_tent);
  hipFree(m->adj_chunk);
  hipFree(m->adj_cspan);
  hipFree(m->jsched);
  delete m;
}

int chem_mech_sizes(const chem_mech* m, int32_t* K, int32_t* R) {
  if (!m) return fail(CHEM_EINVAL, "null mechanism");
  if (K) *K = m->d.K;
  if (R) *R = m->d.R;
  return CHEM_OK;
}

int chem_set_arrhenius(chem_mech* m, const double* lnA, const double* b, const double* theta, void* stream) {
  if (!m || !lnA || !b || !theta) return fail(CHEM_EINVAL, "null argument");
  if (m->d.R == 0) return CHEM_OK;
  hipLaunchKernelGGL(k_set_arrhenius, dim3((m->d.R + 255) / 256), dim3(256), 0, (hipStream_t)stream, m->blob, m->d,
                     m->perm, lnA, b, theta);
  HIPCHK(hipGetLastError());
  return CHEM_OK;
}

static int fill_common(const chem_mech* m, const chem_options* opt, IntArgs& a) {
  chem_options o{};
  o.method = 0;
  o.max_steps = 100000;
  o.fac_safe = 0.9;
  o.fac_min = 0.2;
  o.fac_max = 6.0;
  o.h_min = 1e-20;
  if (opt) o = *opt;
  if (o.method < 0 || o.method > 2) return fail(CHEM_EINVAL, "method must be 0 (ROS4), 1 (Rodas3) or 2 (Seulex)");
  if (o.method == 2 && (o.jac_mode || o.lu_pivot))
    return fail(CHEM_EUNSUPPORTED, "the Seulex integrator uses the analytic Jacobian and pivoted LU");
  if (o.max_steps < 1 || !(o.fac_min > 0.0) || !(o.fac_max >= 1.0) || !(o.fac_safe > 0.0) || !(o.h_min >= 0.0))
    return fail(CHEM_EINVAL, "invalid controller options");
  a.method = o.method;
  a.q = o.method == 1 ? 3.0 : 4.0;
  a.ctl.max_steps = o.max_steps;
  a.ctl.fac_safe = o.fac_safe;
  a.ctl.fac_min = o.fac_min;
  a.ctl.fac_max = o.fac_max;
  a.ctl.h_min = o.h_min;
  if ((o.jac_mode != 0 && o.jac_mode != 1) || (o.lu_pivot != 0 && o.lu_pivot != 1))
    return fail(CHEM_EINVAL, "jac_mode and lu_pivot must be 0 or 1");
  if ((o.jac_mode || o.lu_pivot) && m->wg) return fail(CHEM_EUNSUPPORTED, "ablation switches need N <= 64");
  a.jac_fd = o.jac_mode;
  a.lu_nopiv = o.lu_pivot;
  if (o.fail_lu_lo < 0 || o.fail_lu_hi < o.fail_lu_lo) return fail(CHEM_EINVAL, "need 0 <= fail_lu_lo <= fail_lu_hi");
  a.fail_lu_lo = o.fail_lu_lo;
  a.fail_lu_hi = o.fail_lu_hi;
  return 0;
}

static Variant pick_variant(const chem_mech* m, const chem_options* opt, int64_t ncells) {
  Variant v = m->has_tuned ? m->tuned : Variant{};
  if (!m->has_tuned) v.wpb = max_wpb(m);
  if (opt) {
    if (opt->persistent == 0 || opt->persistent == 1) v.persistent = opt->persistent;
    if (opt->grid_mult > 0) {
      v.grid_mult = opt->grid_mult;
      v.grid_mult_set = true;
    }
    if (opt->jac_slots == -1) {
      v.pool = 0;
    } else if (opt->jac_slots > 0) {
      v.pool = opt->jac_slots;
      v.pool_waves = opt->waves_per_block;  // 0: the most that fit
    }
    if (opt->waves_per_block > 0) {
      v.wpb = opt->waves_per_block;
      if (opt->jac_slots == 0) {
        // a count alone: private Jacobian blocks if they fit, else shared slots
        v.pool = v.wpb <= max_wpb(m) ? 0 : -1;
        v.pool_waves = v.pool ? std::min(v.wpb, 8) : 0;
      }
    }
  }
  v.wpb = std::max(1, std::min(v.wpb, max_wpb(m)));
  (void)ncells;
  return v;
}

int chem_integrate(const chem_mech* mc, int64_t ncells, int64_t ld, double* state, double* h, double p, double dt,
                   double rtol, double atol, const chem_options* opt, int32_t* steps, int32_t* rejects,
                   int32_t* status, void* stream) {
  chem_mech* m = const_cast<chem_mech*>(mc);
  if (!m) return fail(CHEM_EINVAL, "null mechanism");
  if (ncells < 0 || ld < ncells) return fail(CHEM_EINVAL, "need 0 <= ncells <= ld");
  if (ncells == 0) return CHEM_OK;
  if (!state || !h) return fail(CHEM_EINVAL, "null state or h");
  if (!(p > 0.0) || !(dt > 0.0) || !(rtol >= 0.0) || !(atol >= 0.0) || !std::isfinite(p) || !std::isfinite(dt))
    return fail(CHEM_EINVAL, "need p > 0, dt > 0, rtol >= 0, atol >= 0");
  if (ncells > (int64_t)INT32_MAX) return fail(CHEM_EUNSUPPORTED, "more than 2^31-1 cells");
  IntArgs a = base_args(m);
  if (const int rc = fill_common(m, opt, a)) return rc;
  a.state = state;
  a.ld = ld;
  a.ncells = ncells;
  a.h = h;
  a.p = 10.0 * p;
  a.dt = dt;
  a.rtol = rtol;
  a.atol = atol;
  a.steps = steps;
  a.rejects = rejects;
  a.status = status;
  a.prof = opt ? (unsigned long long*)opt->phase_cycles : nullptr;
  const Variant v = pick_variant(m, opt, ncells);
  hipStream_t s = (hipStream_t)stream;
  const bool ordered = opt && opt->cost_order && steps && v.persistent;
  const chem_refmap* rmp = opt ? opt->refmap : nullptr;
  if (rmp) {
    if ((m->d.K > 0 && !rmp->weight) || std::isnan(rmp->z0) || std::isnan(rmp->z_max) || !(rmp->dT >= 0.0))
      return fail(CHEM_EINVAL, "reference mapping needs a weight array, non-NaN z0 and z_max, and dT >= 0");
    if (!m->rm_buf && hipMalloc(&m->rm_buf, sizeof(unsigned long long) * (m->d.N + 1)) != hipSuccess)
      return fail(CHEM_ENOMEM, "reference-mapping buffer allocation failed");
    if (!rmp->ref_of && m->rm_cap < ncells) {
      hipFree(m->rm_flags);
      m->rm_flags = nullptr;
      m->rm_cap = 0;
      if (hipMalloc(&m->rm_flags, sizeof(int32_t) * ncells) != hipSuccess)
        return fail(CHEM_ENOMEM, "reference-mapping flag allocation failed");
      m->rm_cap = ncells;
    }
  }
  int32_t* ref_of = rmp ? (rmp->ref_of ? rmp->ref_of : m->rm_flags) : nullptr;
  if (rmp && !status) {  // mapped cells copy the reference's status, so one is always kept
    if (m->st_cap < ncells) {
      hipFree(m->st_buf);
      m->st_buf = nullptr;
      m->st_cap = 0;
      if (hipMalloc(&m->st_buf, sizeof(int32_t) * ncells) != hipSuccess)
        return fail(CHEM_ENOMEM, "status buffer allocation failed");
      m->st_cap = ncells;
    }
    status = m->st_buf;
    a.status = status;
  }
  const bool queued = ordered || rmp;
  if (queued && m->order_cap < ncells) {
    hipFree(m->order);
    m->order = nullptr;
    m->order_cap = 0;
    if (hipMalloc(&m->order, sizeof(int32_t) * ncells) != hipSuccess)
      return fail(CHEM_ENOMEM, "cost-order buffer allocation failed");
    m->order_cap = ncells;
  }
  if (queued && !m->order_cnt) {
    if (hipMalloc(&m->order_cnt, sizeof(int) * (2 * NBUCKET + 4)) != hipSuccess)
      return fail(CHEM_ENOMEM, "cost-order counter allocation failed");
  }
  if (queued) a.order = m->order;
  if (rmp) a.nactive = m->order_cnt + 2 * NBUCKET;
  if (m->wg) {
    const int rc = ensure_wg_scratch(m, wg_grid(m, ncells), 2);
    if (rc) return rc;
  }
  auto launch_all = [&](hipStream_t st) -> int {
    int rc = 0;
    if (rmp && (rc = launch_refmap_mark(m, *rmp, ref_of, state, ld, ncells, st))) return rc;
    if (queued && (rc = launch_order(m, ordered ? steps : nullptr, ref_of, ncells, st))) return rc;
    if ((rc = launch_integrate(m, a, v, st))) return rc;
    if (rmp) rc = launch_refmap_apply(m, ref_of, state, ld, ncells, h, steps, rejects, status, st);
    return rc;
  };
  if (opt && opt->use_graph && v.persistent) {
    GraphKey key;
    key.v = {(uintptr_t)state, (uintptr_t)h, (uintptr_t)ncells, (uintptr_t)ld, (uintptr_t)steps,
             (uintptr_t)rejects, (uintptr_t)status, (uintptr_t)s, (uintptr_t)v.wpb, (uintptr_t)v.grid_mult,
             (uintptr_t)ordered, (uintptr_t)m->order, (uintptr_t)m->wg_scr, (uintptr_t)m->order_cnt,
             (uintptr_t)(rmp != nullptr), (uintptr_t)(rmp ? rmp->weight : nullptr), (uintptr_t)ref_of,
             (uintptr_t)m->rm_buf, (uintptr_t)a.prof, (uintptr_t)a.ctl.max_steps, (uintptr_t)v.persistent};
    // every value baked into the captured kernel arguments is part of the key
    double dv[14] = {p, dt, rtol, atol, (double)(opt ? opt->method : 0), (double)a.jac_fd, (double)a.lu_nopiv,
                     rmp ? rmp->z0 : 0.0, rmp ? rmp->z_max : 0.0, rmp ? rmp->dT : 0.0,
                     a.ctl.fac_safe, a.ctl.fac_min, a.ctl.fac_max, a.ctl.h_min};
    for (double x : dv) {  // bit patterns (distinguishes -0.0 and NaN payloads too)
      uint64_t u;
      std::memcpy(&u, &x, 8);
      key.v.push_back((uintptr_t)u);
    }
    if (!m->gexec || key.v != m->gkey.v) {
      if (m->gexec) { hipGraphExecDestroy(m->gexec); m->gexec = nullptr; }
      if (m->graph) { hipGraphDestroy(m->graph); m->graph = nullptr; }
      // capture on the library's own stream (the legacy default stream cannot
      // be captured), launch the instantiated graph on the caller's stream
      if (!m->cap_stream) HIPCHK(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc = launch_all(m->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(m->cap_stream, &g);
      if (rc) return rc;
      if (e != hipSuccess) return fail(CHEM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      m->graph = g;
      HIPCHK(hipGraphInstantiate(&m->gexec, g, nullptr, nullptr, 0));
      m->gkey = key;
    }
    HIPCHK(hipGraphLaunch(m->gexec, s));
    return CHEM_OK;
  }
  return launch_all(s);
}

int chem_integrate_noalloc(const chem_mech* mc, int64_t ncells, int64_t ld, double* state, double* h, double p,
                           double dt, double rtol, double atol, const chem_options* opt, int32_t* steps,
                           int32_t* rejects, int32_t* status, void* stream) {
  chem_mech* m = const_cast<chem_mech*>(mc);
  if (!m) return fail(CHEM_EINVAL, "null mechanism");
  if (ncells < 0 || ld < ncells) return fail(CHEM_EINVAL, "need 0 <= ncells <= ld");
  if (ncells == 0) return CHEM_OK;
  if (!state || !h) return fail(CHEM_EINVAL, "null state or h");
  if (!(p > 0.0) || !(dt > 0.0) || !(rtol >= 0.0) || !(atol >= 0.0) || !std::isfinite(p) || !std::isfinite(dt))
    return fail(CHEM_EINVAL, "need p > 0, dt > 0, rtol >= 0, atol >= 0");
  if (ncells > (int64_t)INT32_MAX) return fail(CHEM_EUNSUPPORTED, "more than 2^31-1 cells");
  if (m->wg)
    return fail(CHEM_EUNSUPPORTED, "the no-allocation entry point covers N <= 64 (the workgroup path needs "
                                   "two N x N matrices of scratch per workgroup)");
  if (opt && opt->refmap) return fail(CHEM_EUNSUPPORTED, "no reference-cell mapping in the no-allocation entry point");
  if (opt && opt->use_graph) return fail(CHEM_EINVAL, "the no-allocation entry point keeps no graphs (capture it instead)");
  if (!m->noalloc_scr) return fail(CHEM_EHIP, "device scratch address unavailable");
  IntArgs a = base_args(m);
  if (const int rc = fill_common(m, opt, a)) return rc;
  a.state = state;
  a.ld = ld;
  a.ncells = ncells;
  a.h = h;
  a.p = 10.0 * p;
  a.dt = dt;
  a.rtol = rtol;
  a.atol = atol;
  a.steps = steps;
  a.rejects = rejects;
  a.status = status;
  a.prof = opt ? (unsigned long long*)opt->phase_cycles : nullptr;
  const Variant v = pick_variant(m, opt, ncells);
  hipStream_t s = (hipStream_t)stream;
  const bool ordered = opt && opt->cost_order && steps && v.persistent;
  if (ordered && ncells > NOALLOC_MAX_ORDER)
    return fail(CHEM_EINVAL, "cost-ordered queue of " + std::to_string(ncells) + " cells exceeds the device scratch ("
                                 + std::to_string(NOALLOC_MAX_ORDER) + " cells)");
  int* queue = reinterpret_cast<int*>(m->noalloc_scr);
  if (ordered) {
    int32_t* order = reinterpret_cast<int32_t*>(m->noalloc_scr + NOALLOC_ORDER_OFF);
    int* cnt = reinterpret_cast<int*>(m->noalloc_scr + NOALLOC_CNT_OFF);
    if (const int rc = launch_order(m, steps, nullptr, ncells, s, order, cnt)) return rc;
    a.order = order;
  }
  return launch_integrate(m, a, v, s, queue);
}

int chem_rhs(const chem_mech* m, int64_t ncells, int64_t ld, const double* state, double p, double* f,
             void* stream) {
  if (!m || !state || !f) return fail(CHEM_EINVAL, "null argument");
  if (ncells < 0 || ld < ncells || !(p > 0.0)) return fail(CHEM_EINVAL, "invalid sizes or pressure");
  if (ncells == 0) return CHEM_OK;
  IntArgs a = base_args(m);
  a.ld = ld;
  a.ncells = ncells;
  a.p = 10.0 * p;
  if (m->wg) return launch_rhs_jac_wg(const_cast<chem_mech*>(m), a, state, f, nullptr, (hipStream_t)stream);
  const int wpb = std::max(1, std::min(4, max_wpb(m)));
  const size_t lds = m->d.lds_bytes + (size_t)wpb * cell_bytes(m->d);
  return with_np(m->d.N, [&](auto npc) -> int {
    constexpr int NP = decltype(npc)::value;
    if (set_lds_limit<NP>((const void*)k_rhs_jac<NP>, lds)) return CHEM_EHIP;
    hipLaunchKernelGGL(k_rhs_jac<NP>, dim3((ncells + wpb - 1) / wpb), dim3(wpb * WAVE), lds, (hipStream_t)stream, a,
                       state, f, (double*)nullptr);
    HIPCHK(hipGetLastError());
    return 0;
  });
}

int chem_jacobian(const chem_mech* m, int64_t ncells, int64_t ld, const double* state, double p, double* J,
                  double* f, void* stream) {
  if (!m || !state || !J) return fail(CHEM_EINVAL, "null argument");
  if (ncells < 0 || ld < ncells || !(p > 0.0)) return fail(CHEM_EINVAL, "invalid sizes or pressure");
  if (ncells == 0) return CHEM_OK;
  IntArgs a = base_args(m);
  a.ld = ld;
  a.ncells = ncells;
  a.p = 10.0 * p;
  if (m->wg) return launch_rhs_jac_wg(const_cast<chem_mech*>(m), a, state, f, J, (hipStream_t)stream);
  const int wpb = std::max(1, std::min(4, max_wpb(m)));
  const size_t lds = m->d.lds_bytes + (size_t)wpb * cell_bytes(m->d);
  return with_np(m->d.N, [&](auto npc) -> int {
    constexpr int NP = decltype(npc)::value;
    if (set_lds_limit<NP>((const void*)k_rhs_jac<NP>, lds)) return CHEM_EHIP;
    hipLaunchKernelGGL(k_rhs_jac<NP>, dim3((ncells + wpb - 1) / wpb), dim3(wpb * WAVE), lds, (hipStream_t)stream, a,
                       state, f, J);
    HIPCHK(hipGetLastError());
    return 0;
  });
}

// Workgroup LU (64 < n <= 256): one matrix per 256-thread workgroup, an
// NP x NP scratch slot each; solves (LU == NULL) or writes the factors.
static int lu_wg_launch(int64_t nmat, int32_t n, const double* A, double* b, int32_t* info, double* LU,
                        int32_t* ipiv, void* stream) {
  const int NP = ((n + 15) / 16) * 16;
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = (int)std::min<int64_t>(nmat, std::max(ncu, 1));
  double* scr = nullptr;
  if (hipMalloc(&scr, sizeof(double) * (size_t)grid * NP * NP) != hipSuccess)
    return fail(CHEM_ENOMEM, "LU scratch allocation failed");
  const size_t lds = (size_t)wg_ws_doubles(0, NP, 0) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_lu_wg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_lu_wg, dim3(grid), dim3(WG), lds, (hipStream_t)stream, nmat, n, A, b, info, scr, NP, LU,
                       ipiv);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  hipFree(scr);
  if (e != hipSuccess) return fail(CHEM_EHIP, std::string("workgroup LU: ") + hipGetErrorString(e));
  return CHEM_OK;
}

int chem_lu_solve(int64_t nmat, int32_t n, const double* A, double* b, int32_t* info, void* stream) {
  if (nmat < 0 || n < 1) return fail(CHEM_EINVAL, "need nmat >= 0 and n >= 1");
  if (nmat == 0) return CHEM_OK;
  if (!A || !b || !info) return fail(CHEM_EINVAL, "null argument");
  if (n > 256) return fail(CHEM_EUNSUPPORTED, "n > 256");
  if (n > 64) return lu_wg_launch(nmat, n, A, b, info, nullptr, nullptr, stream);
  return with_np(n, [&](auto npc) -> int {
    constexpr int NP = decltype(npc)::value;
    hipLaunchKernelGGL(k_lu_solve<NP>, dim3((nmat + 3) / 4), dim3(256), 0, (hipStream_t)stream, nmat, n, A, b, info);
    HIPCHK(hipGetLastError());
    return 0;
  });
}

int chem_lu_factor(int64_t nmat, int32_t n, const double* A, double* LU, int32_t* ipiv, int32_t* info,
                   void* stream) {
  if (nmat < 0 || n < 1) return fail(CHEM_EINVAL, "need nmat >= 0 and n >= 1");
  if (nmat == 0) return CHEM_OK;
  if (!A || !LU || !ipiv || !info) return fail(CHEM_EINVAL, "null argument");
  if (n > 256) return fail(CHEM_EUNSUPPORTED, "n > 256");
  if (n > 64) return lu_wg_launch(nmat, n, A, nullptr, info, LU, ipiv, stream);
  return with_np(n, [&](auto npc) -> int {
    constexpr int NP = decltype(npc)::value;
    hipLaunchKernelGGL(k_lu_factor<NP>, dim3((nmat + 3) / 4), dim3(256), 0, (hipStream_t)stream, nmat, n, A, LU,
                       ipiv, info);
    HIPCHK(hipGetLastError());
    return 0;
  });
}

int chem_failed_count(const chem_mech* m, int64_t* out, void* stream) {
  if (!m || !out) return fail(CHEM_EINVAL, "null argument");
  unsigned long long v = 0;
  HIPCHK(hipMemcpyAsync(&v, m->failed, sizeof(v), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  *out = (int64_t)v;
  return CHEM_OK;
}

// Variant <-> the option fields that select it.
static void variant_options(const Variant& v, chem_options& o) {
  o.persistent = v.persistent;
  o.waves_per_block = v.pool > 0 ? v.pool_waves : v.wpb;
  o.grid_mult = v.grid_mult;
  o.jac_slots = v.pool > 0 ? v.pool : -1;
}
static void variant_out(const chem_mech* m, const Variant& v, int32_t* out) {
  out[0] = v.persistent;
  out[1] = m->wg ? 4 : (v.pool > 0 ? v.pool_waves : v.wpb);
  out[2] = v.grid_mult;
  out[3] = m->wg ? 0 : (v.pool > 0 ? v.pool : -1);
}

// The candidate launch variants of a mechanism (every one computes the same bits).
static std::vector<Variant> tune_candidates(const chem_mech* m) {
  std::vector<Variant> c;
  auto add = [&](int persistent, int wpb, int gm, int pool, int pool_waves) {
    Variant v;
    v.persistent = persistent;
    v.wpb = wpb;
    v.grid_mult = gm;
    v.grid_mult_set = true;
    v.pool = pool;
    v.pool_waves = pool_waves;
    c.push_back(v);
  };
  if (m->wg) {
    const int per_cu = std::max(1, (int)(m->max_lds / wg_lds_bytes(m)));
    for (int g = 1; g <= per_cu; ++g) add(1, 4, g, 0, 0);
    return c;
  }
  for (int w = 1; w <= max_wpb(m); ++w) {  // private Jacobian blocks
    add(0, w, 1, 0, 0);
    add(1, w, 1, 0, 0);
    add(1, w, 2, 0, 0);
  }
  if (np_for(m->d.N) > 16) {  // shared Jacobian slots
    for (int w = max_wpb(m) + 1; w <= 8; ++w)
      for (int sl = 2; sl <= std::min(4, w); ++sl) {
        if (pool_lds(m, w, sl) > (size_t)m->max_lds) continue;
        add(1, w, 1, sl, w);
        add(1, w, 2, sl, w);
      }
  }
  return c;
}

int chem_autotune(chem_mech* m, int64_t ncells, int64_t ld, const double* state, const double* h, double p,
                  double dt, double rtol, double atol, int32_t* out_variant, double* out_ms, void* stream) {
  if (!m || !state || !h) return fail(CHEM_EINVAL, "null argument");
  if (ncells < 1 || ld < ncells) return fail(CHEM_EINVAL, "need 1 <= ncells <= ld");
  const int N = m->d.N;
  hipStream_t s = (hipStream_t)stream;
  double *st = nullptr, *hh = nullptr;
  if (hipMalloc(&st, sizeof(double) * N * ncells) != hipSuccess || hipMalloc(&hh, sizeof(double) * ncells) != hipSuccess) {
    hipFree(st);
    return fail(CHEM_ENOMEM, "autotune scratch allocation failed");
  }
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  const std::vector<Variant> cands = tune_candidates(m);
  Variant best = cands.front();
  double best_ms = 1e300;
  int rc = 0;
  chem_options o{};
  o.method = 0;
  o.max_steps = 100000;
  o.fac_safe = 0.9;
  o.fac_min = 0.2;
  o.fac_max = 6.0;
  o.h_min = 1e-20;
  for (const Variant& v : cands) {
    variant_options(v, o);
    double ms_best = 1e300;
    for (int rep = 0; rep < 2 && rc == 0; ++rep) {
      hipMemcpy2DAsync(st, sizeof(double) * ncells, state, sizeof(double) * ld, sizeof(double) * ncells, N,
                       hipMemcpyDeviceToDevice, s);
      hipMemcpyAsync(hh, h, sizeof(double) * ncells, hipMemcpyDeviceToDevice, s);
      hipEventRecord(e0, s);
      rc = chem_integrate(m, ncells, ncells, st, hh, p, dt, rtol, atol, &o, nullptr, nullptr, nullptr, s);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms_best = std::min(ms_best, (double)ms);
    }
    if (rc) break;
    if (ms_best < best_ms) {
      best_ms = ms_best;
      best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(st);
  hipFree(hh);
  if (rc) return rc;
  m->tuned = best;
  m->has_tuned = true;
  if (out_variant) variant_out(m, best, out_variant);
  if (out_ms) *out_ms = best_ms;
  return CHEM_OK;
}

int chem_set_variant(chem_mech* m, const int32_t* v) {
  if (!m || !v) return fail(CHEM_EINVAL, "null argument");
  if ((v[0] != 0 && v[0] != 1) || v[2] < 1 || v[2] > 64) return fail(CHEM_EINVAL, "invalid variant");
  Variant x;
  x.persistent = v[0];
  x.grid_mult = v[2];
  x.grid_mult_set = true;
  if (m->wg) {
    const int per_cu = std::max(1, (int)(m->max_lds / wg_lds_bytes(m)));
    if (v[2] > per_cu) return fail(CHEM_EINVAL, "more workgroups per CU than the LDS holds");
    x.persistent = 1;
  } else if (v[3] > 0) {
    if (np_for(m->d.N) <= 16 || v[1] < 1 || v[1] > 8 || v[3] > v[1] || pool_lds(m, v[1], v[3]) > (size_t)m->max_lds)
      return fail(CHEM_EINVAL, "shared-slot variant does not fit this mechanism");
    x.pool = v[3];
    x.pool_waves = v[1];
    x.wpb = max_wpb(m);
  } else {
    if (v[3] != -1 || v[1] < 1 || v[1] > max_wpb(m)) return fail(CHEM_EINVAL, "private-block variant does not fit");
    x.pool = 0;
    x.wpb = v[1];
  }
  m->tuned = x;
  m->has_tuned = true;
  return CHEM_OK;
}

}  // extern "C"

#include "chem_adjoint_host.inc"
