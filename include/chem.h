/*
 * chem.h — C ABI of the MI355X batched stiff-chemistry integrator.
 *
 * Every CFD cell carries the thermochemical state Phi = (T, Y_1..Y_K) at a
 * fixed pressure p, and the library integrates dPhi/dt = f(Phi) (paper,
 * section 2.1, Eq. 1; all K mass fractions are carried, N = K + 1) over one
 * CFD time step dt with an adaptive Rosenbrock method.  Each step uses the
 * analytical Jacobian and a dense LU factorisation and solve of
 * (I/(gamma h) - J) (section 2.3, Eq. 2 is its one-stage special case).
 *
 * Conventions for every entry point:
 *  - Returns 0 on success or a negative CHEM_E* code; chem_last_error() then
 *    describes the failure (thread-local, valid until the next call).
 *  - Per-cell failures never fail a call: they go to status[c].
 *  - Device pointers are HIP device memory owned by the caller; "stream" is a
 *    hipStream_t (NULL = default stream) and every call is asynchronous on it.
 *  - State arrays are SoA: element (i, c) of an [N][ld] array is at
 *    i * ld + c, row 0 = T in K, rows 1..K = mass fractions; ld >= ncells.
 *  - Units: p in Pa, T in K, dt and h in s, Arrhenius constants in mol-cm-s
 *    with theta = Ea/R in K.
 *  - A chem_mech is used by one stream at a time.
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHEM_OK 0
#define CHEM_EINVAL (-1)       /* invalid argument (pointer, size, mechanism data) */
#define CHEM_EHIP (-2)         /* a HIP runtime call failed */
#define CHEM_ENOMEM (-3)       /* device allocation failed */
#define CHEM_EUNSUPPORTED (-4) /* e.g. N or an efficiency list beyond the compiled limits */

/* per-cell status codes */
#define CHEM_CELL_OK 0
#define CHEM_CELL_TOO_MANY_STEPS 1 /* max_steps attempts did not reach dt */
#define CHEM_CELL_STEP_UNDERFLOW 2 /* the step size fell below h_min */
#define CHEM_CELL_SINGULAR 3       /* I/(gamma h) - J stayed singular after 5 halvings of h */
#define CHEM_CELL_NONFINITE 4      /* non-finite state, T <= 0, or non-finite f / J */
#define CHEM_CELL_TAPE_FULL 5      /* adjoint only: more accepted steps than the tape holds */

/* Mechanism in Chemkin form (host arrays, read during chem_load_mechanism only).
 * Rates follow the standard Chemkin definitions that section 2.3 delegates to
 * pyJac: k = exp(lnA) T^b exp(-theta/T); reverse rates from K_c computed with
 * NASA-7 thermo at p_ref = 1 atm; third-body [M] = sum_k eff_rk C_k; Troe
 * falloff k = k_inf Pr/(1+Pr) F with Pr = k0 [M] / k_inf. */
typedef struct chem_mech_desc {
  int32_t n_species;   /* K >= 1 */
  int32_t n_reactions; /* R >= 0 */
  const double* W;     /* [K] molar masses, g/mol */
  const double* nasa7; /* [K][15]: Tmid, low-range a1..a7, high-range a1..a7 */
  const int32_t* rtype;/* [R] 0 elementary, 1 third-body, 2 Troe falloff */
  const int32_t* reac; /* [R][3] reactant species per molecule slot, -1 = empty */
  const int32_t* prod; /* [R][3] product species per molecule slot, -1 = empty */
  const double* lnA;   /* [R] */
  const double* b;     /* [R] */
  const double* theta; /* [R] Ea/R in K */
  const double* eff;   /* [R][K] third-body efficiencies (ignored for type 0) */
  const double* troe;  /* [R][4] alpha, T***, T*, T** (type 2 only) */
  const double* low;   /* [R][3] lnA0, b0, theta0 of k0 (type 2 only) */
  int32_t n_elements;  /* E >= 0; 0 skips the element-balance check */
  const int32_t* elem; /* [K][E] atoms of each element per molecule (read when E > 0) */
} chem_mech_desc;

typedef struct chem_mech chem_mech; /* opaque, library-owned */

/* Reference-cell mapping of low-reactivity cells (section 2.2: the chemistry
 * solution of one reference cell is mapped onto cells of an ambient zone
 * instead of integrating each; the paper gives no criterion, this one is the
 * library's):
 *  - a cell is in the zone if z = z0 + sum_k weight[k] Y_k <= z_max (summed in
 *    species order with fused multiply-adds; a fuel mass fraction or Bilger's
 *    mixture fraction are such linear indicators);
 *  - the reference is the zone cell of lowest index; it is integrated;
 *  - a zone cell whose T is within dT of the reference's is mapped: not
 *    integrated, it takes the reference's increment per unit mass,
 *    Phi(dt) = Phi(0) + (Phi_ref(dt) - Phi_ref(0)), the reference's h and
 *    status, and zero steps and rejects (also when the reference failed);
 *  - every other cell is integrated as without mapping.
 * The decisions are exact (no tolerance): they are taken in FP64 on the input
 * state in the order stated. */
typedef struct chem_refmap {
  const double* weight; /* device [K], caller-owned, read during the call */
  double z0;            /* indicator offset */
  double z_max;         /* zone threshold (not NaN) */
  double dT;            /* temperature window in K (>= 0; +inf maps the whole zone) */
  int32_t* ref_of;      /* NULL, or device [ncells] out: the reference's index for a
                           mapped cell, -1 for an integrated one */
} chem_refmap;

/* Integrator options; pass NULL for the defaults in brackets. */
typedef struct chem_options {
  int32_t method;     /* 0 ROS4 [0], 1 Rodas3, 2 Seulex-family extrapolated linearly implicit
                         Euler (the paper's integrator; step-number sequence 1..6,
                         order chosen by work per unit step; J frozen per step) */
  int32_t max_steps;  /* step attempts per cell [100000] */
  double fac_safe;    /* step-size safety factor [0.9] */
  double fac_min;     /* smallest step-size ratio [0.2] */
  double fac_max;     /* largest step-size ratio [6] */
  double h_min;       /* step underflow limit in s [1e-20] */
  int32_t persistent; /* -1 auto [-1], 0 one launch slot per cell, 1 persistent grid + work queue */
  int32_t waves_per_block; /* cells per workgroup, 0 = auto [0] */
  int32_t grid_mult;  /* persistent grid = CUs x grid_mult workgroups, 0 = auto [0] */
  int32_t cost_order; /* 1: the persistent queue hands out cells by descending step count,
                         read from steps[] on entry (the previous call's counts; any
                         values are valid, they only set the order); ignored when steps
                         is NULL or the launch is not persistent [0] */
  int32_t use_graph;  /* 1: launch the reset + integrate sequence as a cached hipGraph [0] */
  uint64_t* phase_cycles; /* NULL [NULL], or device [ncells][8] shader-clock cycles per cell:
                             Jacobian pass, forming M, LU, stage f, solves, total, and the
                             reaction and species parts of the Jacobian pass; with method 2
                             slots 6 and 7 count the LU factorisations and the linearly
                             implicit Euler substeps instead */
  /* Ablation switches of section 2.3 (N <= 64; they select the instrumented kernel): */
  int32_t jac_mode;   /* 0 analytic Jacobian [0], 1 one-sided finite differences, column j
                         from f(y + d_j e_j), d_j = sqrt(eps) max(|y_j|, 1e-10) */
  int32_t lu_pivot;   /* 0 partial pivoting [0], 1 no pivoting (rows in natural order) */
  const chem_refmap* refmap; /* NULL [NULL], or reference-cell mapping for this call
                                (chem_integrate only; the adjoint rejects it) */
  int32_t jac_slots;  /* N <= 64, Rosenbrock methods: 0 auto [0]; -1 every wave keeps its own
                         Jacobian block in LDS; n > 0 the workgroup's waves share n Jacobian
                         slots (a wave holds one from its Jacobian pass until M is formed,
                         so more cells fit in a CU's LDS).  With N > 64, grid_mult is the
                         number of workgroups per CU (0: as many as LDS allows). */
  int64_t fail_lu_lo, fail_lu_hi; /* testing [0, 0]: cells with index in [fail_lu_lo, fail_lu_hi)
                         see every factorisation of M as singular (a zero pivot), so the
                         controller's singular branch runs: the step is halved and retried,
                         and the sixth consecutive singular attempt of a step ends the cell
                         with CHEM_CELL_SINGULAR, its state at the step start and h_out the last
                         attempted step size.  CHEM_EINVAL unless 0 <= lo <= hi. */
} chem_options;

/* Validates and uploads the mechanism; *out receives a handle to release with
 * chem_free_mechanism.  Checks (CHEM_EINVAL, message naming the item): species
 * indices in range, positive finite W, finite NASA-7 data with cp > 0 on
 * [200, 6000] K, and, when n_elements > 0, that every reaction conserves each
 * element (sum over reactant molecules of elem = sum over product molecules;
 * the third body M is not a species), as every elementary reaction of the
 * Chemkin form of section 2.1 does.  EUNSUPPORTED if K > 254 or a reaction has
 * more than 8 non-unit efficiencies. */
int chem_load_mechanism(const chem_mech_desc* desc, chem_mech** out);
void chem_free_mechanism(chem_mech* mech);

/* Largest N the compiled kernels accept (255), and the mechanism's sizes.
 * N <= 64 runs one cell per wavefront; 64 < N <= 255 runs one cell per
 * 256-thread workgroup with a blocked LU (chem_integrate_adjoint then returns
 * CHEM_EUNSUPPORTED, and chem_autotune has a single variant to report). */
int chem_max_n(void);
int chem_mech_sizes(const chem_mech* mech, int32_t* K, int32_t* R);

/* Replace lnA, b, theta (device arrays of length R in the order of the
 * descriptor); stream-ordered.  Used to differentiate with respect to them. */
int chem_set_arrhenius(chem_mech* mech, const double* lnA, const double* b, const double* theta,
                       void* stream);

/* Integrate every cell over [0, dt] in place (section 2.1, Eq. 1, with the
 * adaptive Rosenbrock step of section 2.3).
 *  state  : device [N][ld] in/out.
 *  h      : device [ncells] in/out step size; a value <= 0 or non-finite means
 *           start with dt; on return the controller's last unclipped proposal,
 *           capped at dt (the sub-step that persists between CFD steps).
 *  steps, rejects, status : device [ncells] int32 outputs, each may be NULL.
 *  rtol, atol : error control, err = rms(e_i / (atol + rtol max|y_i|)).
 * Uses the library's cached hipGraph when opt->use_graph is 1. */
int chem_integrate(const chem_mech* mech, int64_t ncells, int64_t ld, double* state, double* h, double p,
                   double dt, double rtol, double atol, const chem_options* opt, int32_t* steps,
                   int32_t* rejects, int32_t* status, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * integration of chem_integrate, same arguments, same kernels and the same
 * results bit for bit, with every scratch buffer it needs (the persistent
 * work cursor, the cost-order bucket counters and the cost-ordered queue) in a
 * 2 MiB device array of the library, one per GPU, held until the process ends
 * (its address is looked up once per device by chem_load_mechanism).  No
 * device memory is allocated or freed.  Limits: N <= 64 (CHEM_EUNSUPPORTED
 * above: the workgroup path needs per-workgroup matrices); a cost-ordered
 * queue (opt->cost_order with steps) of at most 524,032 cells (CHEM_EINVAL
 * beyond); no reference-cell mapping (CHEM_EUNSUPPORTED) and no library-owned
 * graph (opt->use_graph: CHEM_EINVAL).  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents: calls that overlap on one
 * GPU (on different streams, or from several threads) race and must not be
 * issued. */
int chem_integrate_noalloc(const chem_mech* mech, int64_t ncells, int64_t ld, double* state, double* h, double p,
                           double dt, double rtol, double atol, const chem_options* opt, int32_t* steps,
                           int32_t* rejects, int32_t* status, void* stream);

/* Number of cells that ended with a nonzero status (CHEM_CELL_*) in the last
 * chem_integrate, chem_integrate_noalloc or chem_integrate_adjoint call on
 * this mechanism that integrated at least one cell (counted on the device also when the call's
 * status pointer was NULL; cells mapped onto a failed reference cell count).
 * Section 2.1: every cell's ODE is solved independently, so a failed cell
 * never fails the call; this reports how many did.  Copies one device counter
 * into *out (host) and synchronises the stream. */
int chem_failed_count(const chem_mech* mech, int64_t* out, void* stream);

/* Discrete adjoint of chem_integrate (not in the paper): integrates forward
 * recording the accepted step sizes and a checkpoint every checkpoint_every
 * accepted steps, then sweeps the Rosenbrock steps backwards with those step
 * sizes frozen.
 *  state0       : device [N][ld] initial states (read only).
 *  lambda_final : device [N][ld] dPsi/dPhi(dt) per cell.
 *  state_final  : device [N][ld] output, may equal neither input.
 *  lambda0      : device [N][ld] output dPsi/dPhi(0), may be NULL.
 *  grad         : device [3][R] output (d/dlnA, d/db, d/dtheta) summed over
 *                 cells in a fixed order (bitwise reproducible).
 *  status       : device [ncells] int32, may be NULL (CHEM_CELL_TAPE_FULL if a
 *                 cell needs more than max_tape accepted steps).
 *  max_tape     : accepted steps recorded per cell (0 = 4096). */
int chem_integrate_adjoint(const chem_mech* mech, int64_t ncells, int64_t ld, const double* state0, double* h,
                           double p, double dt, double rtol, double atol, const chem_options* opt,
                           const double* lambda_final, double* state_final, double* lambda0, double* grad,
                           int32_t checkpoint_every, int32_t max_tape, int32_t* steps, int32_t* status,
                           void* stream);

/* Upper bound, in bytes, of the per-step records that chem_integrate_adjoint
 * keeps for the backward walk of a checkpoint segment (every lane's factor
 * row, pivot step, 1/U_kk and stage values: ncells x checkpoint_every x
 * (NP + 6) x 64 doubles, NP = N rounded up to 16, 32, 56 or 64; device memory
 * owned by the library).  When the records would exceed it, the backward walk
 * replays every step from the segment's states instead: slower, the same
 * results bit for bit.  Default 8 GiB; 0 turns the records off.  Process-wide,
 * for later calls; returns CHEM_OK. */
int chem_set_adjoint_record_budget(uint64_t bytes);

/* Parity entry points for the individual steps of the method.
 * chem_rhs      : f(Phi) of every cell, f is device [N][ld] (Eq. 1).
 * chem_jacobian : J = df/dPhi of every cell, J is device [ncells][N][N]
 *                 row-major (section 2.3, analytical Jacobian); f may be NULL.
 * chem_lu_solve : for each of nmat matrices A (device [nmat][n][n] row-major,
 *                 not modified) solves A x = b in place (b device [nmat][n]),
 *                 LU with partial pivoting as LAPACK getrf/getrs (section 2.3);
 *                 info[m] = 0 or the 1-based step of a zero pivot; n <= 256
 *                 (n > 64 uses the workgroup LU and synchronises the stream). */
int chem_rhs(const chem_mech* mech, int64_t ncells, int64_t ld, const double* state, double p, double* f,
             void* stream);
int chem_jacobian(const chem_mech* mech, int64_t ncells, int64_t ld, const double* state, double p, double* J,
                  double* f, void* stream);
int chem_lu_solve(int64_t nmat, int32_t n, const double* A, double* b, int32_t* info, void* stream);

/* chem_lu_factor: the factorisation alone, in LAPACK getrf's form (section 2.3
 * replaces OpenFOAM's LU with LAPACK's): for each A (device [nmat][n][n]
 * row-major, not modified), LU (device [nmat][n][n] row-major, distinct from A)
 * receives P A = L U with the unit-lower L below the diagonal and U on and
 * above it, and ipiv (device [nmat][n] int32, 0-based like
 * scipy.linalg.lu_factor) the row interchanged with row k at step k.  The
 * pivot of step k is the row of largest |a| among rows k..n-1 in getrf's
 * current order, the first of them on exact ties (idamax).  info as for
 * chem_lu_solve; when info != 0, LU and ipiv are unspecified.  n <= 256 (n > 64
 * synchronises the stream). */
int chem_lu_factor(int64_t nmat, int32_t n, const double* A, double* LU, int32_t* ipiv, int32_t* info,
                   void* stream);

/* The autotuner: times the launch variants on the given input (on a scratch
 * copy; the caller's arrays are not modified) and stores the fastest as the
 * default of this mechanism (used when an option is left at 0).  Variants:
 * N <= 64: private Jacobian blocks (one to four cells per workgroup) or shared
 * Jacobian slots (five to eight cells per workgroup, two to four slots, as the
 * LDS holds them), persistent queue (grid 1 or 2 x CUs) or one launch slot per
 * cell; N > 64: one or two workgroups per CU.  out_variant (host int32[4], may
 * be NULL) receives {persistent, waves_per_block, grid_mult, jac_slots} as in
 * chem_options; out_ms (host, may be NULL) the winner's time.  Every variant
 * computes the same results bit for bit. */
int chem_autotune(chem_mech* mech, int64_t ncells, int64_t ld, const double* state, const double* h, double p,
                  double dt, double rtol, double atol, int32_t* out_variant, double* out_ms, void* stream);

/* Installs a variant as the mechanism's default (for a variant stored from an
 * earlier chem_autotune): variant = host int32[4] {persistent, waves_per_block,
 * grid_mult, jac_slots}.  CHEM_EINVAL if it does not fit this mechanism (too
 * many waves or slots for the LDS, out-of-range values). */
int chem_set_variant(chem_mech* mech, const int32_t* variant);

/* Thread-local description of the last failure. */
const char* chem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHEM_H */
