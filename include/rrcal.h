/*
 * rrcal -- calibrated O(N log N) FFT-correlator for a redundant array on a
 * regular square grid, on AMD Instinct MI355X (gfx950).
 *
 * Method: Gorthi, Parsons & Dillon (2020), "Calibration schemes with
 * O(N log N) scaling for large-N radio interferometers built on a regular
 * grid".  Fig. 1(b) of the paper: channelised antenna voltages feed both an
 * FFT-correlator (gain application, spatial FFT, |.|^2 integrated over time,
 * giving the redundantly averaged visibilities V^unique of eq. modelvis) and
 * a calibrator (a reduced X-engine over a subset of redundant groups giving
 * V^reduced, then redundant-baseline calibration, eq. redcal / eq. redchi,
 * whose gains are applied to the voltages).
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid:   n x n antennas, unit spacing; antenna i sits at (x, y) =
 *         (i mod n, i div n).  N = n*n.
 * Types:  a baseline-type is an integer displacement d = (dx, dy) with
 *         |dx|, |dy| < n in the canonical half-plane (dy > 0, or dy == 0 and
 *         dx > 0).  Its redundant group is every pair (i, j) with
 *         r_i - r_j = d (the orientation of eq. redcal: d_alpha = r_0 - r_1
 *         for V_01); there are N_d = (n - |dx|)(n - |dy|) of them.
 *         `types_xy` arrays hold K such types as 2*K int32 (dx0, dy0, dx1, ...).
 * Pairs:  V^reduced lists the pairs of the selected types type-major, in the
 *         order the types were given; within a type by the raster index of
 *         i.  Pair b of type (dx, dy): with w = n - |dx|, i = (yi, xi) with
 *         yi = b / w + dy, xi = b % w + max(dx, 0), and j = i - (dy*n + dx).
 * Lags:   V^unique holds every canonical lag (2 n (n - 1) of them) in the
 *         order dy ascending, then dx ascending (dy = 0 starts at dx = 1).
 * Units:  one (array, channel) integration.  A plan covers U units of the
 *         same grid; every per-unit array has the unit as its slowest index.
 * Complex numbers are interleaved (re, im); complex64 = two float32.
 *
 * Memory: every pointer argument named `d_*` is device memory owned by the
 * caller (the Python binding allocates it with PyTorch).  The library never
 * allocates device memory; scratch space is the caller's `d_work` buffer of
 * rrc_workspace_size() bytes (no initial contents needed).  A plan owns
 * host memory only.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Device work is enqueued asynchronously; outputs are valid once
 * the stream reaches that point.  A plan (and its workspace) may be used by
 * one stream at a time.
 *
 * Devices: plan creation is host only.  The first call that enqueues device
 * work (or rrc_plan_prepare) binds the plan to the device current then and
 * makes its device resources there: one auxiliary stream and two events
 * (default priority), the device's CU count, the solve kernel's LDS limit.
 * After that, device calls only enqueue kernel launches and event
 * operations, so a caller may capture them into a HIP graph.  Use a plan
 * on the device it is bound to.
 *
 * Errors: every int-returning call returns RRC_OK (0) or a negative code
 * (rrc_strerror() names it).  Invalid arguments are detected on the host
 * before anything is enqueued.  Numerical outcomes of the solve (not
 * converged, non-finite data) never fail a call: they are reported per unit
 * in the `status` output.
 */
#ifndef RRCAL_H
#define RRCAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define RRC_OK        0
#define RRC_EINVAL   -1   /* bad argument (NULL pointer, size, type, mode)   */
#define RRC_EDEGEN   -2   /* selection has more than the four degeneracies  */
#define RRC_EDEVICE  -3   /* a HIP runtime call failed                       */
#define RRC_ENOTIMPL -4   /* combination not supported by this library       */
#define RRC_ERANGE   -5   /* size beyond a documented limit                  */

/* ---- voltage formats ---------------------------------------------------- */
#define RRC_C64 0   /* complex64 samples, 8 bytes                            */
#define RRC_CI4 1   /* 4-bit complex, 1 byte = (re << 4) | (im & 0xF), two's
                       complement nibbles with values in [-7, 7]             */

/* ---- solver options ----------------------------------------------------- */
#define RRC_INIT_FIRSTCAL 0  /* start from logcal amplitudes + chained phases */
#define RRC_INIT_GAINS    1  /* start from the caller's gains                 */
#define RRC_DEGEN_REFANT  0  /* sum ln|g| = 0; antennas (0,0),(1,0),(0,1) real */
#define RRC_DEGEN_MATCH   1  /* match mean ln|g| and the phase plane of g_ref */

/* per-unit solve status */
#define RRC_UNIT_CONVERGED 0
#define RRC_UNIT_MAXITER   1
#define RRC_UNIT_NONFINITE 2

/* Limits of this library. */
#define RRC_MAX_TYPES 16     /* K, selected baseline-types                    */
#define RRC_MAX_GRID  64     /* n; the padded FFT size M <= 128 (rrc_plan_set_fft_size) */

typedef struct rrc_plan rrc_plan;

typedef struct {
    int32_t init_mode;   /* RRC_INIT_*                                            */
    int32_t degen_mode;  /* RRC_DEGEN_*                                           */
    int32_t max_gn;      /* Gauss-Newton steps of the main stage (>= 1)           */
    int32_t fp64_steps;  /* refinement steps after the main stage (>= 0)          */
    int32_t max_cg;      /* CG iterations per normal-equation solve (>= 1)        */
    float   cg_tol;      /* CG stops at ||r|| <= cg_tol ||b|| (sqrt(cg_tol) in    */
                         /* the refinement steps)                                 */
    float   tol32;       /* main stage stops once the rms log-step is below this  */
} rrc_solver_opts;

typedef struct {
    int32_t n;            /* grid side                                   */
    int32_t n_ant;        /* N = n*n                                     */
    int32_t fft_size;     /* M, padded spatial FFT size                  */
    int32_t n_lags;       /* 2 n (n - 1), length of V^unique per unit    */
    int32_t n_types;      /* K                                           */
    int32_t n_pairs;      /* P, length of V^reduced per unit             */
    int32_t dof;          /* P - N - K + 2 (eq. dof)                     */
    int32_t n_units;      /* U                                           */
    int32_t n_time;       /* T, samples per integration                  */
    int32_t dtype;        /* RRC_C64 or RRC_CI4                          */
    uint64_t workspace_bytes;
    int32_t n_live;       /* antennas (N, or the mask's count)           */
    int32_t masked;       /* plan made by rrc_plan_create_masked         */
} rrc_plan_info;

/* Default solver options (FIRSTCAL, REFANT, at most 12 main steps, tol32
 * 1e-5, 1 refinement step, 400 CG iterations, cg_tol 1e-2).  Every step
 * takes its residual and right-hand side in FP64 and solves the normal
 * equations in FP32 (iterative refinement), so the error after a main step
 * is about cg_tol times the step's size, and a refinement step (CG to
 * sqrt(cg_tol)) divides what is left by about 1/sqrt(cg_tol). */
void rrc_default_opts(rrc_solver_opts* opts);

/* Subset redundant-calibration selection (Sec. 5.1, Sec. 5.5
 * eq. subredcal_frac_bls, Sec. 6.1): whole redundant groups in ascending
 * baseline length (ties: dy, then dx), the prefix whose pair count is
 * closest to p N log_b N (ties to the shorter prefix), extended until the
 * degeneracy criterion of Sec. 5.2 holds.  Host only, pure.
 * Writes K types to `types_xy` (room for `cap` types) and K, P to the outputs.
 * log_base <= 1 selects the natural logarithm.  RRC_ERANGE if cap < K. */
int rrc_select_subset(int32_t n, double p, double log_base, int32_t* types_xy,
                      int32_t cap, int32_t* k_out, int32_t* n_pairs_out);

/* Null-space dimension of the linearised calibration system for a
 * selection (Sec. 5.2): amplitude part (ln|g|, ln|V|) and phase part
 * (arg g, arg V).  A valid selection has 1 + 3 = 4.  Host only, pure. */
int rrc_degeneracy_count(int32_t n, const int32_t* types_xy, int32_t k,
                         int32_t* n_null_amp, int32_t* n_null_phase);

/* Predicted gain variance of a selection (Sec. 2 gain uncertainty: eq. cov
 * with eq. noisecov, read per antenna as eq. gaincov / eq. gaincov_v1 of
 * Sec. 5.4): var_out[i] = E|g_i,est / g_i,true - 1|^2 for visibilities of
 * signal-to-noise ratio `snr`, after the degeneracies are fixed the way
 * gains are compared with the truth (mean log-amplitude, and a phase plane
 * c + k.r, removed).  The logarithmic system splits into an amplitude and
 * a phase half, each with noise variance snr^-2 / 2 per equation, so
 * var_out = (snr^-2 / 2) (diag C_eta + diag C_phi), C the projected gains'
 * block of each half's inverse normal matrix.  Host only, FP64, pure;
 * var_out holds n*n doubles.  RRC_EDEGEN for a selection with more than
 * the four degeneracies. */
int rrc_gain_variance(int32_t n, const int32_t* types_xy, int32_t k, double snr, double* var_out);

/* Create a plan for U units of an n x n grid with T samples each.  The
 * selection must satisfy the degeneracy criterion (else RRC_EDEGEN) and,
 * for RRC_INIT_FIRSTCAL, contain the types (1,0) and (0,1).  opts may be
 * NULL (defaults).  n in [2, RRC_MAX_GRID], K in [1, RRC_MAX_TYPES].
 * RRC_ENOTIMPL if a selected type reaches more than 248 antennas back in
 * raster order (dy n + dx > 248), or for RRC_CI4 when n*n is not a
 * multiple of 4 (the X-engine stages whole 32-bit words of 4-bit samples). */
int rrc_plan_create(rrc_plan** out, int32_t n, const int32_t* types_xy, int32_t k,
                    int32_t n_units, int32_t n_time, int32_t dtype,
                    const rrc_solver_opts* opts);
/* ---- masked lattices: hexagonal arrays (Sec. 3, Fig. 2) ------------------
 * An array whose antennas sit on a subset of an n x n lattice index grid:
 * mask[y*n + x] != 0 marks an antenna.  Positions stay integer lattice
 * coordinates, so redundant groups are again equal displacements d and the
 * spatial FFT of the grid (zero where there is no antenna) still gives
 * every lag; only the group sizes N_d change (the mask's autocorrelation).
 * A hexagonal array is the lattice with basis (1, 0), (1/2, sqrt3/2): its
 * axial coordinates (a, b), |a|, |b|, |a + b| < side, sit on the
 * (2 side - 1)^2 grid at (x, y) = (a + side - 1, b + side - 1).
 * Layouts follow the grid: voltages [U][T][n*n] and gains [U][n*n] (values
 * where mask == 0 are never read), V^unique [U][2n(n-1)] with every grid
 * lag (zero at a lag no pair realises), V_auto the mean over the N_live
 * antennas.  V^reduced holds only pairs of two antennas: type-major in the
 * given order, within a type by the raster index of the first antenna.
 * The degeneracy criterion and RRC_DEGEN_REFANT use the first antenna in
 * raster order and its +x and +y neighbours as references (for a full
 * square grid (0,0), (1,0), (0,1)). */
#define RRC_METRIC_SQUARE 0   /* |d|^2 = dx^2 + dy^2                        */
#define RRC_METRIC_HEX    1   /* |d|^2 = dx^2 + dx dy + dy^2 (hex lattice)  */

/* The hexagon of `side` antennas per edge on its (2 side - 1)^2 grid:
 * writes n*n mask bytes (room for `cap`), n and the antenna count
 * (3 side (side - 1) + 1).  Host only, pure. */
int rrc_hex_mask(int32_t side, uint8_t* mask, int32_t cap, int32_t* n_out, int32_t* n_live_out);

/* rrc_select_subset for a masked lattice: types realised by at least one
 * pair, in ascending |d| under `metric` (ties: dy, then dx); group sizes
 * counted over the mask.  Host only, pure. */
int rrc_select_subset_masked(int32_t n, const uint8_t* mask, int32_t metric, double p, double log_base,
                             int32_t* types_xy, int32_t cap, int32_t* k_out, int32_t* n_pairs_out);

/* rrc_degeneracy_count over the mask's antennas and pairs.  Host only. */
int rrc_degeneracy_count_masked(int32_t n, const uint8_t* mask, const int32_t* types_xy, int32_t k,
                                int32_t* n_null_amp, int32_t* n_null_phase);

/* A plan over a masked lattice.  The plan keeps a copy of the mask; every
 * selected type must be realised by a pair, the selection must have the
 * four degeneracies only (else RRC_EDEGEN), and the reference antennas must
 * exist.  Supported calls: rrc_fftcorr, rrc_xengine (dot-product kernel),
 * rrc_omnical, the info/workspace queries, and with RRC_INIT_GAINS (the
 * solve starts from the caller's gains, e.g. the previous integration's)
 * rrc_solve (its d_work is then required), rrc_run and rrc_plan_tune;
 * otherwise those, and rrc_run_static, rrc_chisq_* and batches, return
 * RRC_ENOTIMPL.  Device calls first rebuild the plan's mask, pair and lag
 * tables in d_work from the mask bits the plan passes by value (two small
 * kernels), so the plan still owns no device memory.  Limits as for
 * rrc_plan_create (4-bit plans: n*n a multiple of 4). */
int rrc_plan_create_masked(rrc_plan** out, int32_t n, const uint8_t* mask, const int32_t* types_xy,
                           int32_t k, int32_t n_units, int32_t n_time, int32_t dtype,
                           const rrc_solver_opts* opts);
void rrc_plan_destroy(rrc_plan* plan);
int rrc_plan_get_info(const rrc_plan* plan, rrc_plan_info* info);
int rrc_workspace_size(const rrc_plan* plan, size_t* bytes);

/* Bind the plan to the current device and make its device resources now
 * (see "Devices" above); idempotent. */
int rrc_plan_prepare(rrc_plan* plan);

/* Order of the pipelined run's two branches (see rrc_run):
 * RRC_ORDER_XENG_FIRST (default): X-engine, then the FFT-correlator forked
 *   beside the solve -- for FFT stages that are short or HBM-bound;
 * RRC_ORDER_FFT_FIRST: the FFT-correlator forked first, the X-engine and
 *   the solve beside it -- for a VALU-bound FFT stage that dominates;
 * RRC_ORDER_SERIAL: X-engine, FFT-correlator and solve one after another on
 *   `stream` -- for stages that each fill the device, which slow each other
 *   down more than they gain when they share its CUs.
 * Results are identical in every order. */
#define RRC_ORDER_XENG_FIRST 0
#define RRC_ORDER_FFT_FIRST  1
#define RRC_ORDER_SERIAL     2
int rrc_plan_set_order(rrc_plan* plan, int32_t order);

/* X-engine kernel of a 4-bit plan (complex64 plans have one):
 * RRC_XENG_AUTO (default): the faster form, which on MI355X is the
 *   dot-product one (the matrix-core form keeps one entry per selected
 *   diagonal of each tile and is bound by LDS bank conflicts and its
 *   operand expansion: 27.8 against 9.5 ms at 64x64 x 1024 channels x 4096
 *   samples);
 * RRC_XENG_DOT: signed 4-bit dot products on the vector ALUs;
 * RRC_XENG_MFMA: int8 matrix-core tiles over windows covering the selected
 *   diagonals (RRC_ENOTIMPL if the selection's cover fits none of its
 *   instantiations).  Both are exact; V^reduced is identical bit for bit. */
/* Padded spatial FFT size M of the FFT-correlator (Sec. 1; any M >= 2n - 1
 * gives the same lags, since the padding only keeps the circular
 * correlation from wrapping).  The default is the smallest of 16, 32, 48,
 * 64, 96, 128 with M >= 2n - 1: 48 = 3 x 16 for 17 <= n <= 24 and
 * 96 = 3 x 32 for 33 <= n <= 48 (mixed radix), a power of two otherwise.
 * Where the default is mixed radix, the next power of two (64 or 128) is
 * accepted too; the workspace holds either.  V^unique differs between the
 * two only by FP32 rounding.  RRC_EINVAL for any other size. */
int rrc_plan_set_fft_size(rrc_plan* plan, int32_t fft_size);

#define RRC_XENG_AUTO 0
#define RRC_XENG_DOT  1
#define RRC_XENG_MFMA 2
int rrc_plan_set_xengine(rrc_plan* plan, int32_t kind);

/* (a1)-(a3) FFT-correlator (Fig. 1(b) yellow box; Sec. 2 eq. modelvis).
 * d_volt:   [U][T][N] voltages (complex64, or 1 byte each for RRC_CI4).
 * d_gains:  [U][N] complex64 gains g; the voltages are divided by them.
 * d_vunique:[U][n_lags] complex64, V(d) = C(d) / (N_d T) with C the
 *           time-integrated autocorrelation of the calibrated voltage grid
 *           (the convolution theorem, Sec. 1), equal to eq. modelvis.
 * d_vauto:  [U] float32, C(0) / (N T).  */
int rrc_fftcorr(rrc_plan* plan, void* stream, const void* d_volt, const void* d_gains,
                void* d_vunique, float* d_vauto, void* d_work);

/* (a4) Reduced X-engine (Fig. 1(b) blue box): for every selected pair,
 * V_ij = (1/T) sum_t v_i(t) conj(v_j(t)) on the raw voltages.
 * d_vred: [U][P] complex64 for RRC_C64; for RRC_CI4 [U][P][2] int32 exact
 * raw sums (no 1/T). */
int rrc_xengine(rrc_plan* plan, void* stream, const void* d_volt, void* d_vred, void* d_work);

/* (a5) Reduced redundant calibration (eq. redcal, eq. redchi, eq. dof):
 * minimise chi^2 = sum_b |V_b - g_i conj(g_j) V_alpha|^2 over the gains and
 * the K model visibilities, then fix the four degeneracies (Sec. 5.2).
 * d_vred:      [U][P] as written by rrc_xengine for this plan's dtype.
 * d_gains_in:  [U][N] complex64 start gains (RRC_INIT_GAINS) or NULL.
 * d_gains_ref: [U][N] complex64 reference gains (RRC_DEGEN_MATCH) or NULL.
 * d_gains_out: [U][N] complex64; d_vmodel: [U][K] complex64 (in the units
 *              of d_vred); d_chisq [U] float32 (computed in FP64);
 *              d_niter [U] int32 Gauss-Newton steps; d_status [U] int32. */
int rrc_solve(rrc_plan* plan, void* stream, const void* d_vred, const void* d_gains_in,
              const void* d_gains_ref, void* d_gains_out, void* d_vmodel, float* d_chisq,
              int32_t* d_niter, int32_t* d_status, void* d_work);

/* (a5) The same calibration by omnical's damped simultaneous updates (Sec. 3:
 * the solver of the paper's simulations, damping 0.3): each single g_i and
 * V_alpha is replaced by its exact least-squares minimiser with the others
 * held, blended x <- x + 0.3 (x' - x), until ||x_new - x|| / ||x_new|| < tol
 * (FP32 state; the finishing call fixes the degeneracies like
 * RRC_DEGEN_REFANT and sums chi^2 in FP64).  It is the plain form the
 * adjoint-driven Gauss-Newton solve is measured against.
 * d_vred:     [U][P] as written by rrc_xengine for this plan's dtype.
 * d_gains_in: [U][N] start gains (V_alpha from the group means), or NULL to
 *             continue from the state in d_gains / d_vmodel.
 * max_iter:   iterations of this call (per unit; a unit stops when
 *             converged).  One call per iteration with d_delta read back is
 *             the host-stepped form; one call with many the device form.
 * finish:     non-zero: degeneracy fix, chi^2 and final status.
 * d_gains [U][N], d_vmodel [U][K]: complex64 state in, result out;
 * d_niter [U]: iterations so far (set by a call with d_gains_in, else
 * increased); d_status [U]: RRC_UNIT_*; d_delta [U] (optional): the last
 * relative change; d_chisq [U] (finish only).
 * d_work: the plan's workspace, required for a masked plan (its pair
 * tables), may be NULL otherwise.  A masked plan's grid points without an
 * antenna keep gain 0 and take no part. */
int rrc_omnical(rrc_plan* plan, void* stream, const void* d_vred, const void* d_gains_in, int32_t max_iter,
                float tol, int32_t finish, void* d_gains, void* d_vmodel, float* d_chisq, int32_t* d_niter,
                int32_t* d_status, float* d_delta, void* d_work);

/* (a5) chi^2 only: d_chisq[u] = sum_b |V_b - g_i conj(g_j) V_alpha|^2 for
 * complex64 d_g [U][N], d_vm [U][K], d_vred [U][P] (complex64, any dtype
 * plan; int sums must be converted by the caller).  FP32 products, FP64 sum. */
int rrc_chisq_fwd(rrc_plan* plan, void* stream, const void* d_g, const void* d_vm,
                  const void* d_vred, float* d_chisq);

/* (a6) Adjoint of chi^2 (from eq. redchi): the gradient in PyTorch's complex
 * convention, 2 d chi^2 / d conj(z), for z = g ([U][N]) and z = V ([U][K]):
 *   2 dchi2/dconj(g_i) = -2 [ sum_{(i,j)} r_b g_j conj(V_a) + sum_{(k,i)} conj(r_b) g_k V_b' ]
 *   2 dchi2/dconj(V_a) = -2 sum_{b in a} r_b conj(g_i) g_j
 * with r_b = V_b - g_i conj(g_j) V_alpha, and the diagonal of J^H J:
 *   diag_g_i = sum_{(i,j)} |g_j V_a|^2 + sum_{(k,i)} |g_k V_b'|^2,
 *   diag_v_a = sum_{b in a} |g_i g_j|^2.
 * Outputs complex64 d_grad_g [U][N], d_grad_v [U][K], float32 d_diag_g
 * [U][N], d_diag_v [U][K]; any output pointer may be NULL to skip it. */
int rrc_chisq_adj(rrc_plan* plan, void* stream, const void* d_g, const void* d_vm,
                  const void* d_vred, void* d_grad_g, void* d_grad_v, float* d_diag_g,
                  float* d_diag_v);

/* The whole hot path for one integration of U units.
 * mode RRC_RUN_PIPELINED: the FFT-correlator applies d_gains_in (the
 *   previous integration's solution, Fig. 1 real-time loop) while the
 *   X-engine and the solve run on the same voltages; the solved gains are
 *   for the next integration.  The FFT-correlator runs on the plan's
 *   auxiliary stream, forked from `stream` after the X-engine (or before it,
 *   see rrc_plan_set_order) and joined back into it with events, so all
 *   outputs are ordered on `stream` as usual.  d_gains_out may be the same
 *   buffer as d_gains_in (the loop feeding its solution back): the FFT then
 *   reads a copy of the gains taken in the workspace before the solve.
 * mode RRC_RUN_SELFCAL: X-engine, solve, then the FFT-correlator applies the
 *   just-solved gains (reads the voltages twice).
 * Outputs as in the calls above; d_gains_in may be NULL in SELFCAL mode.
 * d_stamps (optional, may be NULL): [1 + U] uint64 device-clock stamps --
 *   d_stamps[0] when the run starts on the device, d_stamps[1 + u] when the
 *   last of unit u's outputs (solve, V^unique) is written; ticks of the
 *   constant-rate wall clock, rrc_wall_clock_hz() per second. */
#define RRC_RUN_PIPELINED 1
#define RRC_RUN_SELFCAL   2
typedef struct {
    const void* d_volt;
    const void* d_gains_in;
    const void* d_gains_ref;
    void*    d_vunique;
    float*   d_vauto;
    void*    d_vred;
    void*    d_gains_out;
    void*    d_vmodel;
    float*   d_chisq;
    int32_t* d_niter;
    int32_t* d_status;
    void*    d_work;
    uint64_t* d_stamps;
} rrc_io;
int rrc_run(rrc_plan* plan, void* stream, int32_t mode, const rrc_io* io);

/* rrc_run without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid allocation).  Identical to rrc_run except that io->d_work must be
 * NULL: the scratch space is a static device array of the library,
 * RRC_STATIC_SCRATCH_BYTES per GPU (held until the process ends), whose
 * address is looked up once per device (hipGetSymbolAddress) when a plan
 * is bound to it.  The plan must be prepared first (rrc_plan_prepare, or
 * any earlier device call: the set-up that makes its stream and events and
 * looks the address up), else RRC_EINVAL; the call itself creates and
 * allocates nothing, it only enqueues launches and event operations.
 * RRC_ERANGE when the plan's
 * rrc_workspace_size() exceeds RRC_STATIC_SCRATCH_BYTES (e.g. the 16x16
 * grid with 64 channels and 1024 samples needs about 20 MB; larger plans
 * use rrc_run).  Every plan on one GPU shares that GPU's one array, which
 * keeps the last call's contents (no call needs them cleared): calls that
 * overlap in time on one GPU -- on different streams, or different plans --
 * race on it and must be ordered by the caller. */
#define RRC_STATIC_SCRATCH_BYTES (32u << 20)
int rrc_run_static(rrc_plan* plan, void* stream, int32_t mode, const rrc_io* io);

/* ---- low-cadence calibration (Sec. 4) -----------------------------------
 * The calibrator correlates about p N log N baselines at a time (the budget
 * of eq. lowcadcal_inttime) and cycles through every redundant group, whole
 * groups per cycle, so N_cycle cycles of t_int = t_cal / N_cycle populate
 * the full visibility matrix, which is then calibrated once over every
 * type.  Groups are taken in V^unique's lag order; a cycle takes whole
 * groups while its pair count stays within p N ln N (log_base as in
 * rrc_select_subset).  The populated matrix is the all-type pair list: the
 * types in lag order, each type's pairs in the raster order of the first
 * antenna (the layout of V^reduced with every type selected), P = N(N-1)/2. */
#define RRC_LOWCAD_MAX_GRID   32    /* n of the low-cadence entry points        */
#define RRC_LOWCAD_MAX_CYCLES 256

/* The round robin: cycle c correlates lag-order types
 * [type_begin[c], type_begin[c+1]); type_begin gets n_cycles + 1 entries
 * (room for `cap`).  Host only, pure. */
int rrc_lowcad_schedule(int32_t n, double p, double log_base, int32_t* type_begin, int32_t cap,
                        int32_t* n_cycles);

/* The populated matrix: d_volt [U][T][N] complex64 voltages of one
 * calibration interval; cycle c integrates samples
 * [floor(c T / n_cycles), floor((c+1) T / n_cycles)), and each pair's entry
 * is the mean of v_i conj(v_j) over its cycle's samples (FP32).
 * d_vfull: [U][N(N-1)/2] complex64.  n <= RRC_LOWCAD_MAX_GRID,
 * n_cycles <= RRC_LOWCAD_MAX_CYCLES <= T. */
int rrc_lowcad_xengine(int32_t n, int32_t n_units, int32_t n_time, const int32_t* type_begin,
                       int32_t n_cycles, void* stream, const void* d_volt, void* d_vfull);

/* Redundant calibration of the populated matrix over every type by
 * omnical's damped updates (as rrc_omnical, finished: degeneracies fixed
 * like RRC_DEGEN_REFANT, chi^2 in FP64), starting from d_gains_in (the
 * previous interval's solution) with V_alpha from the group means.
 * d_gains [U][N], d_vmodel [U][2n(n-1)] complex64 (lag order); d_chisq,
 * d_niter, d_status [U].  3 <= n <= RRC_LOWCAD_MAX_GRID. */
int rrc_lowcad_solve(int32_t n, int32_t n_units, void* stream, const void* d_vfull, const void* d_gains_in,
                     int32_t max_iter, float tol, void* d_gains, void* d_vmodel, float* d_chisq,
                     int32_t* d_niter, int32_t* d_status);

/* Whole-array goodness of fit (Sec. 2: the reduced calibration's gains and
 * the FFT-correlator's V^unique, eq. modelvis, against the full visibility
 * matrix of an FX correlator; the metric of Sec. 6.4): for every pair of the
 * all-type list, r_ij = V_ij - g_i conj(g_j) V^unique(d_ij), and per unit
 * d_chisq[u] = sum |r_ij|^2 (eq. redchi with sigma_ij = 1) and, when
 * d_chisq_cal is not NULL, d_chisq_cal[u] = sum |r_ij / (g_i conj(g_j))|^2
 * (residuals of the calibrated visibilities, whose sample noise is the same
 * for every pair).  Both FP64.  d_vfull: [U][N(N-1)/2] complex64, the
 * all-type list (e.g. rrc_lowcad_xengine with one cycle); d_gains [U][N],
 * d_vunique [U][2n(n-1)] complex64.  n <= RRC_LOWCAD_MAX_GRID. */
int rrc_chisq_full(int32_t n, int32_t n_units, void* stream, const void* d_vfull, const void* d_gains,
                   const void* d_vunique, double* d_chisq, double* d_chisq_cal);

/* Autotuner of a plan's launch parameters for the pipelined run on this
 * device: the FFT-correlator's time chunk (1, 2 or 4 times the default
 * length, i.e. fewer workgroups each integrating more samples and fewer
 * partial grids for the finish), the branch order (rrc_plan_set_order) and,
 * for 4-bit plans whose cover fits, the X-engine kernel
 * (rrc_plan_set_xengine), and the FFT size (rrc_plan_set_fft_size) where a
 * second one fits.  Each candidate runs the whole path (rrc_run,
 * PIPELINED, on `io`, whose contents it overwrites) once to warm up and
 * three times under HIP events on `stream`; the fastest is applied to the
 * plan.  cache_path (may be NULL): a text file of past choices, one line
 * per device (architecture, CU count) and plan shape (grid, types, U, T,
 * dtype); a matching line is applied without timing, a new choice is
 * appended.  Synchronises `stream`; not for use under graph capture.
 * V^reduced and the solve's outputs are identical for every candidate;
 * V^unique differs only by the order in which the time chunks' partial
 * power grids are added (FP32 rounding). */
typedef struct {
    int32_t fft_chunk_factor;
    int32_t order;      /* RRC_ORDER_*                              */
    int32_t xengine;    /* RRC_XENG_*                               */
    float   ms_per_run; /* the chosen candidate's time per rrc_run */
    int32_t from_cache;
    int32_t fft_size;   /* M (rrc_plan_set_fft_size)                */
} rrc_tune;
int rrc_plan_tune(rrc_plan* plan, void* stream, const rrc_io* io, const char* cache_path, rrc_tune* out);

/* A batch of plans (one per array; grids, channels and sample counts may
 * differ) whose hot paths run together: the uneven-batch case of several
 * arrays calibrated at once (Fig. 1 real-time loop over every channel of
 * every array).  The plans must be distinct and outlive the batch.  Host
 * only; owns streams and events.
 * flags: 0.  RRC_BATCH_GRAPH (replaying the whole batch as one captured
 * graph launch) returns RRC_ENOTIMPL in this library: capturing the batch's
 * fork/join ended the process with a host-side fault in the runtime. */
#define RRC_BATCH_GRAPH 1u
typedef struct rrc_batch rrc_batch;
int rrc_batch_create(rrc_batch** out, int32_t n_plans, rrc_plan* const* plans, uint32_t flags);
void rrc_batch_destroy(rrc_batch* batch);

/* rrc_run(plans[i], ..., mode, &io[i]) for every plan, in one call on
 * `stream`: each plan runs on its own branch stream (owned by the batch,
 * made at the first run on the current device, default priority), forked
 * from `stream` and joined back into it with events, so the arrays run
 * concurrently and all outputs are ordered on `stream`.  With more units in
 * the batch than compute units the solves share CUs.
 * Asynchronous like rrc_run; one batch may be run by one stream at a time,
 * and its plans must not be run concurrently on other streams. */
int rrc_batch_run(rrc_batch* batch, void* stream, int32_t mode, const rrc_io* io);

/* Ticks per second of the device wall clock that d_stamps count (current
 * device). */
int rrc_wall_clock_hz(double* hz);

const char* rrc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* RRCAL_H */
