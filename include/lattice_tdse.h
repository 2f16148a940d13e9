/*
 * lattice_tdse.h -- C-ABI of the MI355X Strang-splitting library.
 *
 * Method: Suzuki, Suryanarayana, Nuyens, "Strang splitting in combination
 * with rank-1 and rank-r lattices for the time-dependent Schroedinger
 * equation" (arXiv:1808.06357).  The library advances
 *
 *     i gamma du/dt = -(gamma^2/2) lap u + v(x) u,   x in [0,1)^d periodic,
 *
 * (Sec. 1, eq. (TDSE)) on the points of a rank-1 or rank-2 lattice with the
 * Strang scheme of eq. (StrangTDSE) / Algorithm 1, on one AMD GPU.
 *
 * Conventions shared by every call:
 *   - A lattice (Def. 1) is given by r generating vectors z_1..z_r in Z^d,
 *     stored row-wise: Z[i*d + j] = j-th component of z_i, and moduli
 *     n_1..n_r with n_{i+1} | n_i.  N = n_1 * ... * n_r.
 *   - Point index kappa = sum_i k_i prod_{j>i} n_j (Sec. 2.5, last index
 *     fastest); point p_kappa = (sum_i z_i k_i / n_i) mod 1.
 *   - Frequency key chi(h) = sum_i xi_i prod_{j>i} n_j with
 *     xi_i = h.z_i mod n_i (Def. 2, Thm. 1(iii), Sec. 2.5).
 *   - The state u is the vector of lattice values u(p_kappa) in kappa order
 *     (equivalent to the coefficient vector of Algorithm 1 through the
 *     unitary DFT of eqs. (Fnx)/(Fn): uhat = F u / sqrt(N)).
 *   - Complex data are interleaved (re, im): LT_C64 = 2 x float,
 *     LT_C128 = 2 x double (the layout of torch.complex64 / complex128).
 *   - One step: u <- P u; U = F u; U <- K U; u = F^{-1} U; u <- P u with
 *     P = diag(exp(-i dt v_kappa / (2 gamma))) and
 *     K = diag(exp(-i 2 pi^2 gamma dt ||h_chi||^2)) (eqs. (Dn), (Vn),
 *     (StrangTDSE)).  The phase arguments are formed and reduced mod 2 pi in
 *     double precision in both precisions.  Prime (chirp-z) lengths run
 *     F^{-1} K F as one zero-padded cyclic convolution (runs of 4 steps or
 *     more); its kernel spectrum is built in double, and LT_C64 runs apply
 *     it rounded once to complex float, like the rest of their arithmetic.
 *
 * Memory: every pointer documented "device" is device memory owned by the
 * caller, who must keep it alive until the work queued on `stream` has
 * finished.  The library never retains a caller pointer.  A plan owns its own
 * host tables and device tables and frees them in lattice_plan_destroy.
 * Streams are hipStream_t passed as void* (NULL = the default stream).
 *
 * Errors: argument and plan errors are detected on the host before anything
 * is queued and reported through the return value; HIP failures return
 * LT_E_HIP.  lt_last_error() gives a message for the calling thread's last
 * non-OK status.  No call aborts the process or throws across the ABI.
 */
#ifndef LATTICE_TDSE_H
#define LATTICE_TDSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lt_plan lt_plan;

typedef enum { LT_C64 = 1, LT_C128 = 2 } lt_prec;

typedef enum {
    LT_OK = 0,
    LT_E_ARG = 1,            /* bad argument (null pointer, size, value)          */
    LT_E_NOT_CANONICAL = 2,  /* moduli not canonical (Def. 1: n_{i+1} | n_i)     */
    LT_E_NOT_INJECTIVE = 3,  /* index set violates Def. 2                          */
    LT_E_INCOMPLETE = 4,     /* not every key reachable: lattice points not distinct */
    LT_E_NOMEM = 5,
    LT_E_HIP = 6,            /* a HIP runtime call failed (or no GPU)              */
    LT_E_UNSUPPORTED = 7     /* valid input outside what this build implements    */
} lt_status;

/* Read-only facts about a plan. */
typedef struct {
    int32_t d, r;
    int64_t n[4];            /* moduli (first r used)                                */
    int64_t N;               /* number of lattice points = number of keys            */
    int64_t n_index;         /* size of the user index set I (0 if none given)       */
    int64_t n_completed;     /* keys given minimal-l2 representatives (N - |I|)      */
    int64_t max_s;           /* max ||h_chi||^2 over all keys                        */
    int32_t bluestein;       /* 1: the length-N transform runs as a chirp-z convolution */
    int32_t passes;          /* 1: whole run in one workgroup; 2: column + row passes;
                                3: three levels (power-of-two L of 2^24 points or more) */
    int64_t fft_len;         /* transform length L (N, or the convolution length)    */
    int32_t L1, L2;          /* column / row lengths of the two-pass layout (L = L1*L2;
                                up to 4096 x 4096, above that 4096 x 8192 at most);
                                three levels: outer and inner column lengths      */
    int32_t cols;            /* columns per column-pass workgroup                     */
    int32_t rows;            /* rows per row-pass workgroup                           */
    int32_t L3;              /* three levels: row length (L = L1*L2*L3); else 0       */
    int32_t swapped;         /* 1: a rank-2 tensor n1 x n2 whose n1-point columns are
                                long (n1 >= 2048, n2 <= n1/4): strang_run transposes
                                the state and v into the workspace and runs on
                                n2-point columns and n1-point rows (L1, L2 above
                                describe the untransposed layout) */
} lt_plan_info;

/*
 * lattice_plan -- planning of a lattice and its index set.
 *
 * Builds the lattice of Def. 1 and its anti-aliasing set of full
 * cardinality (Def. 2, Thm. 1):
 *   - H (nh x d, row-major int32, may be NULL with nh = 0) is a user index
 *     set; it must be injective under chi (LT_E_NOT_INJECTIVE otherwise) and
 *     its elements own their keys;
 *   - complete = 1: every key not owned by H gets its minimal-l2
 *     representative (Lemma 4, eq. (hrepresenter)), ties broken by h
 *     lexicographic (h_1 first, signed ascending), found with the
 *     construction of Sec. 3.1 (enumerate a ball, sort by norm, first unseen
 *     key wins); complete = 0: H must own all N keys (|H| = N), otherwise
 *     LT_E_INCOMPLETE; H = NULL always plans the minimal-l2 full set;
 *   - prec_mask: 0 plans on the host only (no GPU needed; each run builds
 *     the device tables of its precision on first use); LT_C64 and / or
 *     LT_C128 also build the device tables a forward run in those precisions
 *     reads, on the calling thread's current device (LT_E_HIP without one),
 *     so that later runs with a workspace allocate nothing.
 * Requirements: 1 <= r <= 2 for runs (planning accepts r <= 4), d >= 1,
 * n_{i+1} | n_i (LT_E_NOT_CANONICAL), all N points distinct
 * (LT_E_INCOMPLETE; for rank-1 this is gcd(N, z_1..z_d) = 1).
 * Components of z_i sharing a factor with n_i are accepted when the points
 * stay distinct, which is the property Thm. 1 uses.
 * On success *out owns the plan; release it with lattice_plan_destroy.
 */
lt_status lattice_plan(int32_t d, int32_t r, const int64_t *Z, const int64_t *n,
                       const int32_t *H, int64_t nh, int32_t complete, int32_t prec_mask,
                       lt_plan **out);

/* Copy the plan's facts into *info. */
lt_status lattice_plan_info(const lt_plan *p, lt_plan_info *info);

/*
 * Host copies of the plan's integer tables (for bit-exact checks); each
 * output may be NULL.  key_of_h: chi(h) for each row of the H given at
 * planning (nh entries); s_of_key: ||h_chi||^2 (N entries);
 * h_of_key: h_chi (N x d, row-major).
 */
lt_status lattice_plan_keys(const lt_plan *p, int64_t *key_of_h, int64_t *s_of_key,
                            int32_t *h_of_key);

/*
 * Lattice points (Def. 1) as exact integer numerators: for kappa in
 * [first, first + count), num[(kappa-first)*d + j] = (sum_i z_{i,j} k_i N/n_i) mod N,
 * so that p_kappa = num / N.  Host memory.
 */
lt_status lattice_plan_points(const lt_plan *p, int64_t first, int64_t count, int64_t *num);

void lattice_plan_destroy(lt_plan *p);

/*
 * Bytes of device workspace strang_run needs for (p, prec, batch,
 * shared_v) -- shared_v = 1 when v_stride == 0.  Written to *bytes.
 */
lt_status strang_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, int32_t shared_v,
                                size_t *bytes);

/*
 * strang_run -- m Strang steps (eq. (StrangTDSE); Algorithm 1) for `batch`
 * independent states on one lattice, in place.
 *   v      device, double, N values per state in kappa order (the diagonal
 *          of V_n, eq. (Vn)); state b uses v + b * v_stride (v_stride = 0
 *          shares one potential).
 *   u      device, batch x N complex of `prec`: in u(0), out u(m dt).
 *   gamma  > 0, the scaled Planck constant of eq. (TDSE); dt any real (a
 *          negative dt runs the scheme backwards: S(-dt) = S(dt)^{-1}).
 *   steps  >= 0.
 *   ckpt   optional (NULL with ckpt_every = 0): device, complex of `prec`,
 *          ceil(steps / ckpt_every) x batch x N; receives u at steps
 *          0, K, 2K, ... (K = ckpt_every), layout [c][b][kappa].
 *   work   device workspace of at least strang_workspace_size bytes, or NULL
 *          (then the call allocates and frees it stream-ordered).
 * Successive half potential steps are merged into one full step, which
 * equals the literal scheme within rounding.
 * A rank-2 plan with lattice_plan_info.swapped = 1 runs on the transposed
 * tensor: u and v are transposed into the workspace, stepped there and u is
 * transposed back; checkpoints are stored in kappa order (the caller's
 * buffers stay in kappa order; the result equals the untransposed run
 * within rounding).
 * With `work` given, and once an earlier call on the plan and precision has
 * built the plan's device tables, the call enqueues kernel launches (and,
 * with checkpoints, one device-to-device copy) on `stream` and nothing else:
 * no allocation, memset or synchronisation, so a caller can capture it into
 * a HIP graph and replay it.
 */
lt_status strang_run(const lt_plan *p, lt_prec prec, int32_t batch, const double *v,
                     int64_t v_stride, void *u, double gamma, double dt, int64_t steps,
                     void *ckpt, int64_t ckpt_every, void *work, size_t work_bytes, void *stream);

/*
 * strang_run_noalloc -- strang_run (same arguments, no checkpoints) for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The run's workspace is a static
 * device array of the library, one per GPU, held until the process ends; the
 * call allocates nothing (no hipMalloc, no stream-ordered allocation) and
 * only enqueues kernels on `stream`.
 *   - The plan's device tables for `prec` must exist (lattice_plan with prec
 *     in prec_mask, or an earlier run): otherwise LT_E_ARG, before any launch.
 *   - A run whose workspace (strang_workspace_size) exceeds the array
 *     (strang_run_noalloc_capacity: 128 MiB) fails with LT_E_ARG.
 *   - Every call on one GPU shares that GPU's array, and the array keeps the
 *     last call's contents (a run rebuilds everything it reads from it), so
 *     calls that overlap on one GPU (other streams, other threads) race.
 */
lt_status strang_run_noalloc_capacity(size_t *bytes);
lt_status strang_run_noalloc(const lt_plan *p, lt_prec prec, int32_t batch, const double *v,
                             int64_t v_stride, void *u, double gamma, double dt, int64_t steps,
                             void *stream);

/*
 * strang_run_sums -- strang_run (same arguments and semantics) that also
 * records, at every step boundary j = 0..steps, the two point sums of the
 * state u_j of Sec. 3.3 (norm conservation and the potential part of the
 * energy <H u, u>, H = -(gamma/2) Laplacian + v/gamma):
 *   sums[(b (steps+1) + j) 2 + 0] = (1/N) sum_k |u_j(p_k)|^2
 *   sums[(b (steps+1) + j) 2 + 1] = (1/(gamma N)) sum_k v(p_k) |u_j(p_k)|^2
 * (sums: device, batch x (steps+1) x 2 doubles, written by the call).
 * The column pass at each step boundary holds the point values up to a unit
 * phase and forms the tile sums in FP64 as it passes (one extra read of v per
 * point); the partials are reduced in a fixed order, so the result is
 * reproducible run to run.  The kinetic part of the energy needs F u_j, which
 * no pass of a merged step holds: lattice_diagnostics on checkpoints gives it.
 *   work   at least strang_run_sums_workspace_size bytes (which depends on
 *          steps), or NULL.
 */
lt_status strang_run_sums_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch,
                                         int32_t shared_v, int64_t steps, size_t *bytes);
lt_status strang_run_sums(const lt_plan *p, lt_prec prec, int32_t batch, const double *v,
                          int64_t v_stride, void *u, double gamma, double dt, int64_t steps,
                          void *ckpt, int64_t ckpt_every, double *sums, void *work,
                          size_t work_bytes, void *stream);

/*
 * strang_adjoint -- reverse-mode derivative of u(T) = S^m u(0) for a real
 * loss J, for `batch` states sharing the plan (same v, dt, gamma convention
 * as strang_run).  Gradients use g = dJ/dRe + i dJ/dIm.
 *   uT     device, batch x N: u(T) from the forward run.
 *   gT     device, batch x N: dJ/du(T).
 *   ckpt   device, the forward checkpoints of strang_run (required,
 *          ckpt_every >= 1).  The forward states are recomputed by running
 *          the unitary step backwards (S^{-1} = S^H) and reset to the stored
 *          checkpoint every ckpt_every steps to bound drift.
 *   g0     device out, batch x N: dJ/du(0).
 *   gv     device out, double: dJ/dv; N values if v_stride == 0 (summed
 *          over the batch), batch x N otherwise.
 *   work   device workspace of at least strang_adjoint_workspace_size
 *          bytes, or NULL.
 * Per step, with a = P u^{j-1}, b = F^{-1} K F a, y = conj(P) g_j and
 * mu = F^{-1} conj(K) F y, the potential gradient collects
 * dt/(2 gamma) [Im(conj(y) b) + Im(conj(mu) a)] and g_{j-1} = conj(P) mu.
 * A rank-2 plan with a swapped schedule (lattice_plan_info.swapped) sweeps
 * the transposed tensor like its forward run: the workspace then also holds
 * transposed copies of u(T), gT and v; every input and output stays in
 * lattice order.
 */
lt_status strang_adjoint_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch,
                                        int32_t shared_v, size_t *bytes);
lt_status strang_adjoint(const lt_plan *p, lt_prec prec, int32_t batch, const double *v,
                         int64_t v_stride, const void *uT, const void *gT, double gamma, double dt,
                         int64_t steps, const void *ckpt, int64_t ckpt_every, void *g0, double *gv,
                         void *work, size_t work_bytes, void *stream);

/*
 * strang_run_batched -- B independent problems, each with its own plan,
 * potential, state, gamma, dt and step count (eq. (StrangTDSE) for each),
 * advanced together: problems small enough for one workgroup run their whole
 * step loop inside one shared launch; the others are interleaved pass by
 * pass in shared launches.  Arrays are host arrays of length B holding
 * device pointers (v[b]: N_b doubles, u[b]: N_b complex of `prec`, in place).
 *   work   device workspace of at least strang_batched_workspace_size bytes,
 *          or NULL.
 */
lt_status strang_batched_workspace_size(int32_t B, const lt_plan *const *plans, lt_prec prec,
                                        size_t *bytes);
lt_status strang_run_batched(int32_t B, const lt_plan *const *plans, lt_prec prec,
                             const double *const *v, void *const *u, const double *gamma,
                             const double *dt, const int64_t *steps, void *work,
                             size_t work_bytes, void *stream);

/*
 * Batch objects -- the problems of strang_run_batched planned once, for
 * callers that advance the same batch again and again (and may capture the
 * advance into a HIP graph).
 *
 * strang_batch_create takes the arguments of strang_run_batched (same
 * meaning; host arrays of length B holding device pointers).  It allocates
 * the batch's device memory (workspace and descriptor tables), builds every
 * member's kinetic table, merged potential table and chirp-z convolution
 * spectrum from gamma, dt and v on `stream`, and returns once they are built.
 * The object keeps the device pointers v[b] and u[b]: both buffers must stay
 * allocated, and v[b] unchanged, until the object is destroyed.
 *
 * strang_batch_run advances every u[b] in place by steps[b] Strang steps
 * (eq. (StrangTDSE) for each member; the same passes as strang_run_batched).
 * It only enqueues kernels and event operations on `stream`: no allocation,
 * copy, memset or host wait, so it may be captured into a HIP graph, and each
 * replay advances the states once more.  Calls on one object must not overlap
 * (they share the object's workspace).
 *
 * strang_batch_autotune times the register-staged kernel geometries
 * (variants 1, 2 and, for lengths up to 2048, 5 of lattice_plan_set_kernels)
 * of every length class of the batch on scratch copies of the members'
 * buffers (the states are untouched; reps launches per timing, three
 * interleaved rounds of which the fastest counts) and keeps the fastest per
 * class; it synchronizes `stream`.
 * strang_batch_kernels lists the classes: key[i] > 0 is a column class of
 * column length key[i], key[i] < 0 a row class (-key = 2 L2 + multiplier
 * kind), variant[i] its geometry (up to cap entries; *ncls gets the count).
 * strang_batch_destroy waits for the device and frees the object.
 */
typedef struct lt_batch lt_batch;
lt_status strang_batch_create(int32_t B, const lt_plan *const *plans, lt_prec prec,
                              const double *const *v, void *const *u, const double *gamma,
                              const double *dt, const int64_t *steps, void *stream,
                              lt_batch **out);
lt_status strang_batch_run(const lt_batch *b, void *stream);
lt_status strang_batch_autotune(lt_batch *b, int32_t reps, void *stream);
lt_status strang_batch_kernels(const lt_batch *b, int32_t *ncls, int32_t *key, int32_t *variant,
                               int32_t cap);
void strang_batch_destroy(lt_batch *b);

/*
 * lattice_projection_error -- the two key sums of the initial (spatial)
 * discretization error of Sec. 3.4: for a function g with Fourier
 * coefficients ghat(h) and its lattice approximation g_a (coefficients
 * ghat_a(h_xi) = (1/N) sum_k g(p_k) exp(-2 pi i h_xi . p_k) on the index set
 * A = {h_xi}: e_total^2 = ||g||^2 - sum_A |ghat|^2 + sum_A |ghat - ghat_a|^2
 * (the first two terms are the coefficients outside A).  The library forms
 * ghat_a by the lattice DFT of the point values and returns both sums.
 *   u      device, batch x N complex of `prec`: g at the lattice points.
 *   ghat   device, batch x N complex double (interleaved), key order: the
 *          coefficient of g at the plan's representative h_xi of key xi
 *          (lattice_plan_keys h_of_key).
 *   out    device, batch x 2 doubles: (sum_A |ghat|^2, sum_A |ghat - ghat_a|^2).
 *   work   at least lattice_projection_error_workspace_size bytes, or NULL.
 * The transform runs in the precision of u; the sums accumulate in double.
 * Errors: LT_E_ARG (NULL buffers, precision, batch < 0).
 */
lt_status lattice_projection_error_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, size_t *bytes);
lt_status lattice_projection_error(const lt_plan *p, lt_prec prec, int32_t batch, const void *u,
                                   const double *ghat, double *out, void *work, size_t work_bytes,
                                   void *stream);

/*
 * splitting_run -- m steps of a symmetric composition of the Strang step of
 * eq. (StrangTDSE): order 2 is the Strang step itself (as strang_run, in the
 * two-pass layout); order 4 is the triple jump S(w1 dt) S(w0 dt) S(w1 dt) with
 * w1 = 1 / (2 - 2^(1/3)), w0 = 1 - 2 w1 (Yoshida's composition; global error
 * O(dt^4)), the higher-order splitting the paper names as a continuation
 * (Sec. 5).  Consecutive half potential steps are merged.
 *
 * Time-dependent potentials (the other continuation named in Sec. 5):
 * v(x, tau) = v(x) + f(tau) v1(x).  Time advances with the kinetic flow, so
 * a substep of length h from tau applies the potential half steps at tau
 * and at tau + h: exp(-i h v(., tau) / (2 gamma)), F^-1 K(h) F,
 * exp(-i h v(., tau + h) / (2 gamma)).  This is the Strang step of the
 * autonomous system extended by the clock; it keeps order 2, and the triple
 * jump keeps order 4, for smooth f.
 *   v1     device, N doubles per state (strided as v), or NULL for a
 *          time-independent potential.
 *   f      host, m * P + 1 doubles (P = 1 for order 2, 3 for order 4):
 *          f at the substep boundaries tau_j that splitting_times returns,
 *          read during the call; ignored when v1 is NULL.
 * Other arguments as in strang_run (no checkpoints); work: at least
 * splitting_workspace_size bytes, or NULL.  Errors: LT_E_ARG for an order
 * other than 2 or 4, for v1 without f, or non-finite f (and as strang_run);
 * LT_E_UNSUPPORTED for a chirp-z lattice whose complex128 schedule differs
 * from the run's (the convolution spectra are built in double).  Every
 * substep of a chirp-z lattice runs in the convolution form.
 */
lt_status splitting_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, int32_t shared_v,
                                   int32_t order, size_t *bytes);
lt_status splitting_run(const lt_plan *p, lt_prec prec, int32_t batch, const double *v,
                        const double *v1, int64_t v_stride, const double *f, void *u, double gamma,
                        double dt, int64_t steps, int32_t order, void *work, size_t work_bytes,
                        void *stream);

/*
 * splitting_times -- the substep boundaries of an m-step run of
 * splitting_run started at t0: tau[k P + i] = t0 + (k + c_i) dt for
 * k < m, i < P, with c_0 = 0 and c_{i+1} = c_i + w_i, and tau[m P] = t0 + m dt
 * (for order 4 the middle boundaries step backwards, w0 < 0).
 * tau: host, m * P + 1 doubles (caller-owned).  Errors: LT_E_ARG.
 */
lt_status splitting_times(int32_t order, int64_t steps, double t0, double dt, double *tau);

/*
 * lattice_diagnostics -- the conserved quantities of Sec. 3.3 for `batch`
 * states of lattice values u: the L2 norm^2 and the energy <H u, u> with
 * H = -(gamma/2) lap + v/gamma, on the lattice
 *   norm^2 = (1/N) sum_k |u_k|^2,
 *   E      = (1/N) [ sum_xi 2 pi^2 gamma ||h_xi||^2 |U_xi|^2 + (1/gamma) sum_k v_k |u_k|^2 ],
 * U = F u the unitary lattice DFT (eq. (Fn) / (Fnx)), so that uhat = U / sqrt(N)
 * are the coefficients on the anti-aliasing set (Parseval).  The transform runs in
 * the precision of u; every sum accumulates in double.
 *   v      device, N doubles per state (v_stride as in strang_run).
 *   u      device, batch x N complex of `prec` (not modified).
 *   out    device, batch x 2 doubles: (norm^2, E) per state.
 *   work   device workspace of at least lattice_diagnostics_workspace_size
 *          bytes, or NULL.
 * With strang_run's checkpoints as u this gives the norm and energy history
 * of a run (every ckpt_every steps).
 */
lt_status lattice_diagnostics_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch,
                                             size_t *bytes);
lt_status lattice_diagnostics(const lt_plan *p, lt_prec prec, int32_t batch, const double *v,
                              int64_t v_stride, const void *u, double gamma, double *out,
                              void *work, size_t work_bytes, void *stream);

/*
 * Kernel selection for two-pass schedules.  Each column / row pass can run
 * on one of several kernels with identical results (within rounding):
 *   0 = general LDS Stockham kernel (any 7-smooth length),
 *   1 = register-staged kernel, 256 threads x 16 elements (radix 16 / 8),
 *   2 = register-staged kernel, 512 threads x 8 elements (radix 8 / 4),
 *   3 = register-staged kernel with its own tiles: 64 threads x 16
 *       elements (1024-element tiles, four times the workgroups of 1 and 2,
 *       for small transforms), or, for 4096-point columns, 512 threads x 16
 *       elements holding two columns per tile;
 *   4 = 512 threads x 8 elements with twice the registers of variant 2
 *       (two waves per SIMD); a column workgroup takes two tiles, the
 *       second tile's loads in flight while the first is transformed;
 *   5 = 256 threads x 8 elements on 2048-element tiles (twice the
 *       workgroups of 1, 2 and 4, two waves per SIMD).
 * Variants 1 and 2 exist for the power-of-two lengths 64 ... 4096, variant
 * 3 for 64 ... 1024 and 4096-point columns, variant 4 for columns of
 * 64 ... 4096 points and rows of 64 ... 4096, variant 5 for 64 ... 2048;
 * elsewhere the general kernel runs whatever is selected (rows of 8192
 * points always take their own 512-thread kernel).  Variants outside
 * 0 ... 5 give LT_E_ARG.
 * The default is 1, except for complex128 column passes of at most 2048
 * points, which default to 5 (the geometry that holds the step's fused
 * sums of strang_run_sums without spilling registers).
 * A plan keeps two choices per pass: one for launches of a single state (or
 * of few points) and one for launches of many states, batch >= 2 with
 * batch * L >= 2^20 points (L = the schedule's transform length).  A
 * single state's grid fits the chip in one residency wave whose load,
 * compute and store phases run in lockstep; many states give several waves
 * that overlap, and the fastest variant differs between the two.
 * lattice_plan_autotune times every applicable variant of the plan's
 * steady-state column and row passes on `stream`, once on one state and
 * once on max(2, ceil(2^22 / L)) states sharing v (reps launches each, in
 * three interleaved rounds of which the fastest counts, on a scratch buffer
 * it allocates and frees), and keeps the fastest of each class; it must not
 * run concurrently with runs of the same plan.
 * One-workgroup and three-level schedules have nothing to tune (the latter
 * run the default variant 1).
 * lattice_plan_set_kernels sets both classes to the given variants;
 * lattice_plan_get_kernels reports the single-state choice and
 * lattice_plan_get_kernels_batch the choice a launch of `batch` states
 * (batch >= 1) takes.
 */
lt_status lattice_plan_autotune(lt_plan *p, lt_prec prec, int32_t reps, void *stream);
lt_status lattice_plan_set_kernels(lt_plan *p, lt_prec prec, int32_t col_variant, int32_t row_variant);
lt_status lattice_plan_get_kernels(const lt_plan *p, lt_prec prec, int32_t *col_variant,
                                   int32_t *row_variant);
lt_status lattice_plan_get_kernels_batch(const lt_plan *p, lt_prec prec, int32_t batch,
                                         int32_t *col_variant, int32_t *row_variant);

/*
 * Diagnostics: HIP-event timing of the library's own launches.  While
 * enabled, every kernel launch is bracketed by two events recorded on its
 * stream.  lt_timing_enable(on) also discards earlier records;
 * lt_timing_summary waits for the recorded events of one kernel class and
 * returns their count and summed elapsed milliseconds.
 */
typedef enum { LT_KIND_COLUMN = 0, LT_KIND_ROW = 1, LT_KIND_RESIDENT = 2 } lt_kernel_kind;
lt_status lt_timing_enable(int32_t on);
lt_status lt_timing_summary(int32_t kind, int64_t *launches, double *total_ms);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *lt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LATTICE_TDSE_H */
