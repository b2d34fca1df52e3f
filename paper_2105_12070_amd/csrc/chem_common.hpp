// Shared definitions of the HIP path: packed mechanism layout (written by the
// host packer, read by the kernels), Rosenbrock tables, kernel arguments and
// wavefront primitives for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chem {

constexpr double RU = 8.314462618e7;  // gas constant, erg/(mol K)
constexpr double PATM = 1.01325e6;     // standard-state pressure, dyn/cm^2
constexpr int MAXTB = 8;               // non-unit third-body efficiencies per reaction
constexpr int WAVE = 64;

enum CellStatus { ST_OK = 0, ST_TOO_MANY = 1, ST_UNDERFLOW = 2, ST_SINGULAR = 3, ST_NONFINITE = 4, ST_TAPE = 5 };

// Packed mechanism.  Reactions are stored sorted by type: [0,R0) elementary,
// [R0,R1) third-body, [R1,R) Troe.  Empty molecule slots and unused efficiency
// slots point at the padding species index K, whose concentration is 1 and
// whose g/RT and h/RT are 0, so the kernels need no branches for them.
struct MechDims {
  int K, R, N, S;  // species, reactions, N = K+1, LDS row stride of J (odd, >= N+1)
  int R0, R1;      // type boundaries
  int L;           // species->reaction incidence entries
  // byte offsets inside the LDS-staged blob
  int o_lnA, o_b, o_th, o_sp, o_W, o_iW, o_cptr, o_cent;
  int o_tbp, o_tbs, o_tbd, o_troe;  // third-body lists and Troe data
  int lds_bytes;   // size of the staged blob (multiple of 16)
};

// Third-body / Troe reaction r >= R0 has the non-unit efficiencies
// tbs[e], 1 + tbd[e] for e in [tbp[r-R0], tbp[r-R0+1]) (at most MAXTB).
// Troe data per falloff reaction: alpha, 1/T***, 1/T*, T**, lnA0, b0, theta0, 0.
constexpr int TROE_STRIDE = 8;

// Rosenbrock method in the transformed form (Hairer & Wanner IV.7):
//   M = I/(gamma h) - J,  M K_i = f(y + sum_j a_ij K_j) + sum_j (c_ij/h) K_j,
//   y_new = y + sum m_i K_i,  err = sum e_i K_i.
struct RosTable {
  int s;
  int newf[4];      // stage i evaluates f at a point no earlier stage used
  int src[4];       // the stage whose f evaluation stage i uses
  double gamma;
  double a[4][4], c[4][4], m[4], e[4];
};

// 0: ROS4 with Shampine's parameters (as tabulated by Sandu et al. 1997),
// order 4 with an embedded order-3 estimate; 1: Rodas3 (Sandu et al. 1997),
// stiffly accurate, order 3(2).
__constant__ const RosTable kTables[2] = {
    {4, {0, 1, 1, 0}, {0, 1, 2, 2}, 0.57282,
     {{0, 0, 0, 0}, {2.0, 0, 0, 0}, {1.867943637803922, 0.2344449711399156, 0, 0},
      {1.867943637803922, 0.2344449711399156, 0.0, 0}},
     {{0, 0, 0, 0}, {-7.137615036412310, 0, 0, 0}, {2.580708087951457, 0.6515950076447975, 0, 0},
      {-2.137148994382534, -0.3214669691237626, -0.6949742501781779, 0}},
     {2.255570073418735, 0.2870493262186792, 0.4353179431840180, 1.093502252409163},
     {-0.2815431932141155, -0.07276199124938920, -0.1082196201495311, -1.093502252409163}},
    {4, {0, 0, 1, 1}, {0, 0, 2, 3}, 0.5,
     {{0, 0, 0, 0}, {0, 0, 0, 0}, {2.0, 0, 0, 0}, {2.0, 0, 1.0, 0}},
     {{0, 0, 0, 0}, {4.0, 0, 0, 0}, {1.0, -1.0, 0, 0}, {1.0, -1.0, -8.0 / 3.0, 0}},
     {2.0, 0.0, 1.0, 1.0},
     {0.0, 0.0, 0.0, 1.0}}};

struct Controller {
  int max_steps;
  double fac_safe, fac_min, fac_max, h_min;
};

// Arguments of the integration kernels.
struct IntArgs {
  const uint8_t* blob;      // LDS-staged part of the mechanism (global copy)
  const double* nasa;       // [K][16] Tmid, lo a1..a7, hi a1..a7, pad
  const uint32_t* jsched;   // [jsched_it][64] species-scatter schedule of the Jacobian (wavefront path)
  int jsched_it;
  MechDims d;
  int method;               // index into kTables
  double q;                 // controller exponent 1/q (4 ROS4, 3 Rodas3)
  Controller ctl;
  double* state;            // [N][ld]
  int64_t ld, ncells;
  double* h;                // [ncells]
  double p;                 // dyn/cm^2
  double dt, rtol, atol;
  int32_t* steps;
  int32_t* rejects;
  int32_t* status;
  int* queue;               // persistent work cursor (NULL: one cell per wave slot)
  const int32_t* order;     // optional cell order for the queue
  const int* nactive;       // optional device count of queue entries (default ncells)
  int cell_doubles;         // per-wave LDS workspace in doubles
  int pool_slots;           // Jacobian slots shared by the workgroup's waves (0: every wave has its own)
  // adjoint tape (NULL in the forward integrator)
  double* tape_h;           // [ncells][max_tape]
  double* tape_y;           // [ncells][max_tape/ckpt + 1][N]
  int max_tape, ckpt;
  unsigned long long* prof; // [ncells][8] per-phase cycle counts, or NULL
  unsigned long long* failed; // cells that ended with a nonzero status (counter), or NULL
  int64_t fail_lu_lo, fail_lu_hi; // cells in [lo, hi) see every factorisation of M as singular (testing)
  int jac_fd;               // ablation (instrumented kernel only): finite-difference Jacobian
  int lu_nopiv;             // ablation (instrumented kernel only): LU without pivoting
};

// ------------------------------------------------------------ wave primitives
__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ double readlane(double x, int l) {
  unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int uniform_int(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ double uniform_double(double x) { return readlane(x, 0); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

template <unsigned CTRL>
__device__ __forceinline__ unsigned dpp(unsigned x) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
template <unsigned CTRL>
__device__ __forceinline__ double dpp(double x) {
  unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  unsigned lo = dpp<CTRL>((unsigned)u), hi = dpp<CTRL>((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror
constexpr unsigned DPP_QP1032 = 0xB1, DPP_QP2301 = 0x4E, DPP_HMIRROR = 0x141, DPP_MIRROR = 0x140;

// Wave sum in a fixed order: pairwise within each row of 16 lanes (both
// partners add the same two operands, and IEEE addition commutes, so all lanes
// of a row agree bitwise), then the four row sums combined as (r0+r1)+(r2+r3).
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp<DPP_QP1032>(x);
  x += dpp<DPP_QP2301>(x);
  x += dpp<DPP_HMIRROR>(x);
  x += dpp<DPP_MIRROR>(x);
  const double r0 = readlane(x, 0), r1 = readlane(x, 16), r2 = readlane(x, 32), r3 = readlane(x, 48);
  return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned x) {
  x = max(x, dpp<DPP_QP1032>(x));
  x = max(x, dpp<DPP_QP2301>(x));
  x = max(x, dpp<DPP_HMIRROR>(x));
  x = max(x, dpp<DPP_MIRROR>(x));
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)x, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)x, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)x, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)x, 48);
  return max(max(r0, r1), max(r2, r3));
}

// Orders the wave's LDS traffic between phases in which lanes read what
// other lanes wrote.
// Waits until the wave's outstanding LDS operations (atomics without return
// included) have completed: s_waitcnt lgkmcnt(0), the other counters at their
// maximum.  Placed after each loop of LDS atomic accumulations, before the
// sums are read.
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xc07f); }

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace chem
