// Internal declarations shared by the host planner, the C-ABI layer and the
// HIP kernels of the lattice Strang library.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lattice_tdse.h"

namespace lt {

constexpr int kThreads = 256;           // workgroup size of every FFT kernel
constexpr int kMaxStages = 24;
constexpr int64_t kTileElems = 4096;     // complex elements per workgroup tile
constexpr int64_t kWideRow = 8192;       // row length of the widest two-pass split (one row per workgroup)
// dynamic LDS every FFT kernel may request: the 160 KB of a CU less 1 KB for
// the static arrays of the block reductions (static + dynamic must fit)
constexpr int kMaxDynLds = 159 * 1024;

// Radix sequence of one sub-transform of length L (product of radices).
struct Radices {
    int L;
    int n;
    int r[kMaxStages];
};

// How one lattice transform is laid out on the GPU for one precision.
struct Sched {
    bool ok = false;
    int passes = 0;          // 1: one workgroup holds the whole transform; 2: column + row passes
    bool bluestein = false;  // the length-N DFT runs as a chirp-z convolution of length L
    bool rank2 = false;      // 2-D transform over n1 x n2 (no four-step twiddle)
    int64_t L = 0;           // transform length (N, or the convolution length)
    int L1 = 0, L2 = 0;      // two-pass: column length, row length; single rank-2: n1, n2
    int cols = 1;            // columns per column-pass workgroup
    int rows = 1;            // rows per row-pass workgroup
    int ept = 16;            // max complex elements per thread (register budget)
    int col_var = 1;         // column-pass kernel: 0 general, 1 fast 256x16, 2 fast 512x8,
                             // 3 fast 64x16 (1024-element tiles), 4 fast 512x8 with two
                             // waves per SIMD, 5 fast 256x8 (2048-element tiles)
    int row_var = 1;         // row-pass kernel (same codes)
    int col_var_m = 1;       // the same choices for launches of many states
    int row_var_m = 1;       // (see many_states)
    Radices ra{}, rb{};      // radices of L1 (or L) and of L2
    // three-level layout (passes == 3, power-of-two L of at least 2^24 points):
    // L = L1 * L2 * L3; the column pass over L1 takes L2 := L2 * L3 as its row
    // length, the inner column pass runs over L2 (radices rc) inside each of
    // the L1 blocks of L2 * L3 points, and the row pass over L3 (radices rb)
    int L3 = 0;
    int cols2 = 1;           // inner columns per workgroup
    Radices rc{};
    // rank-2 tensor held transposed (n2 x n1): the column pass runs over n2,
    // the row pass over the contiguous n1 (a run's first and last steps
    // transpose the state and the potential)
    bool swapped = false;
};

// A launch over many states fills the chip with several residency waves of
// workgroups, whose load, compute and store phases overlap; a single state's
// grid runs them in lockstep.  The fastest kernel variant differs between the
// two regimes, so a plan keeps one choice for each.
constexpr int64_t kManyPoints = int64_t(1) << 20;
inline bool many_states(const Sched &s, int batch) { return batch > 1 && batch * s.L >= kManyPoints; }
inline int col_variant_of(const Sched &s, int batch) { return many_states(s, batch) ? s.col_var_m : s.col_var; }

// A pass whose working set (the states plus at most 32 bytes of tables per
// transform point) fits the 256 MB Infinity Cache with room to spare stores
// the state with write-through; larger ones keep the write-back L2.
constexpr int64_t kCacheResident = int64_t(192) << 20;
inline bool cache_resident(const Sched &s, int64_t state_bytes, int batch)
{
    return (int64_t)batch * s.L * state_bytes + 32 * s.L <= kCacheResident;
}
inline int row_variant_of(const Sched &s, int batch) { return many_states(s, batch) ? s.row_var_m : s.row_var; }

// Device tables of a plan for one precision (built lazily, then immutable).
struct DevTables {
    bool built = false;
    void *twa = nullptr;     // W_{La}^q, q < La (Tw<T> format), La = L1 or L
    void *twb = nullptr;     // W_{L2}^q
    double *tw4hi = nullptr; // W_L^{qa L2}, qa < L1   (double complex pairs)
    double *tw4lo = nullptr; // W_L^{qb},    qb < L2
    int32_t *s_key = nullptr;// ||h_chi||^2 per key, natural order
    int32_t *s_row = nullptr;// ||h_chi||^2 at the row-pass positions (two-pass, no chirp-z)
    double *bhat = nullptr;  // chirp-z kernel spectrum / (L sqrt N), complex double, schedule layout
    int64_t ktab_n = 0;      // entries of a run's kinetic table (max_s + 1)
    // three-level layout: W_{L2} stage table and the inner four-step twiddles
    // W_M^{q}, M = L2 L3 (hi: qa < L2 in steps of L3, lo: qb < L3)
    void *twc = nullptr;
    double *tw4hi2 = nullptr, *tw4lo2 = nullptr;
};

// ---------------------------------------------------------------- kernel arguments
// Point-domain multiplier of a column pass, at natural index n < Nvalid:
//   w = exp(-i phase v[n]) * ktab[s[n]] * c_n^chirp * scale
// (terms with a null pointer / zero flag are skipped; c_n is the chirp
// exp(-pi i (n^2 mod 2N)/N); ktab[m] = exp(-i kin m) for the integer
// squared norms m = ||h||^2); indices n >= Nvalid are set to zero.
struct ColArgs {
    void *buf; int64_t buf_bs;        // transform buffer (L elements per batch item)
    const void *in; int64_t in_bs;    // first pass: read lattice values from here (Nvalid)
    void *out; int64_t out_bs;        // last pass: write lattice values here (Nvalid)
    int L1, L2, C, ntiles;
    int64_t Nvalid;
    int pre_inv, post_fwd, twiddle;
    const double *v; int64_t v_bs; double phase;
    const double *v2; double phase2; // optional second field: angle phase v[n] + phase2 v2[n]
                                      // (time-dependent potentials; v2 strided as v)
    const int32_t *s; const double *ktab;
    int chirp;                        // +1: times c_n, -1: times conj(c_n), 0: none
    int64_t Nchirp;
    double scale;
    const double *tw4hi, *tw4lo;      // four-step twiddle tables (complex double)
    const void *ptab; int64_t ptab_bs;// merged potential step exp(-i phase v[n]) per point, cx<T>
                                      // (fast passes; the general kernel uses v and phase)
    const void *twa;                  // Tw<T> table of W_{L1}
    Radices rad;
    void *ck; int64_t ck_bs;          // optional checkpoint store of the point value
    const double *ck_v;               // u = x * exp(-i ck_phase ck_v[n]) * conj(c_n)^[ck_chirp]
    double ck_phase;
    int ck_chirp;
    int ck_t;                         // 1: the tile is a transposed rank-2 tensor, point n = k1 L2 + c
                                      // is stored at c L1 + k1 (lattice order)
    // adjoint pairing: sequences of vector 0 (state) and vector 1 (cotangent)
    int adjoint;                      // 0: off; 1: first; 2: middle; 3: last
    void *buf2; int64_t buf2_bs;      // cotangent transform buffer
    const void *in2; int64_t in2_bs;  // first adjoint pass: cotangent lattice values
    void *out2; int64_t out2_bs;      // last adjoint pass: dJ/du0
    double *gacc; int64_t gacc_bs;    // potential gradient accumulator (double, natural index)
    double gcoef;                     // coefficient of Im(conj(mu) a) in the accumulator
    const void *reset; int64_t reset_bs;  // checkpoint replacing the recomputed state, or null
    double reset_phase;               // a = exp(-i reset_phase v) * ckpt (times c_n for chirp-z)
    int reset_t;                      // 1: the tile is a transposed rank-2 tensor whose checkpoints are
                                      // in lattice order: point n = k1 L2 + c reads ckpt[c L1 + k1]
    // per-step sums at a step boundary (the point values x have |x| = |u_j|):
    // sum_part[(b sum_pt + tile) 2 + {0, 1}] = (sum |x|^2, sum sum_v[n] |x|^2)
    // over the tile's valid points; sum_v strided as v (v_bs)
    double *sum_part; int sum_pt;
    const double *sum_v;
    int wt;                           // register-staged passes: store the state with write-through
                                      // (set by launch_col from the launch's working set)
};

// Spectral multiplier of a row pass at row-pass position pos = k1 L2 + k2:
// chirp-z: bhat[pos] (complex double, conjugated if conj_tab);
// otherwise ktab[s[pos]] (kinetic phase per squared norm, 1/L folded in).
struct RowArgs {
    void *buf; int64_t buf_bs;
    int L1, L2, rows, nblk;
    const double *bhat; int conj_tab;
    const float *bhat_f;              // complex64 register-staged rows: the same spectrum rounded once
                                      // to complex float (interleaved pairs), or null
    const int32_t *s; const double *ktab;
    int64_t ktab_n;                   // entries of ktab (its squared-norm range)
    int fft_only;
    const void *twb;                  // Tw<T> table of W_{L2}
    Radices rad;
    int wt;                           // register-staged passes: store the state with write-through
                                      // (set by launch_row from the launch's working set)
};

struct ResArgs {
    void *u; int64_t u_bs;
    int64_t N, L;
    int rank2, n1, n2;
    Radices ra, rb;
    const void *twa, *twb;
    int bluestein;
    const int32_t *s;                  // ||h||^2 per key, natural order
    const double *ktab;                // exp(-i kin m) * (1/L smooth, 1 chirp-z), m = ||h||^2
    const double *bhat;                // natural order, chirp-z only (complex double)
    const double *v; int64_t v_bs;
    double phase_half;                 // dt / (2 gamma)
    int64_t steps;
    void *ck; int64_t ck_every; int64_t ck_stride; // checkpoint c at ck + c*ck_stride + b*N
    int64_t batch;
    double *sum_part;                  // optional: (sum |u_j|^2, sum v |u_j|^2) at ((j batch + b) 2)
};

// One two-pass problem of a batch: its column / row arguments per role and
// the number of passes of its schedule.
struct BatchDesc {
    ColArgs col[4];   // 0 first, 1 potential P^2, 2 kinetic (chirp-z), 3 last
    RowArgs row[2];   // 0 spectral multiplier, 1 conjugated spectrum (chirp-z)
    int64_t npass;    // 2m + 1 (smooth N) or 4m + 1 (chirp-z)
    int bluestein;
    int pad;
};

// kinetic table of one problem of a batch: dst[m] = exp(-i kin m) * scale, m < count
struct KtabDesc {
    double *dst;
    int64_t count;
    double kin, scale;
};

// ---------------------------------------------------------------- launchers (kernels.hip)
// All launchers return 0 or a hipError_t value; they enqueue on `stream`.
int launch_col(int prec, const Sched &s, const ColArgs &a, int batch, void *stream);
int launch_row(int prec, const Sched &s, const RowArgs &a, int batch, void *stream);
int launch_resident(int prec, const Sched &s, const ResArgs &a, int batch, void *stream);
int launch_fft_single(const Radices &ra, const void *twa_c128, void *buf, int64_t L, void *stream);
// per-step sums: hist[b][j0 + j] = (sum of the PT partials of slot j) * (inv_n, inv_gn), j < count
int launch_step_sums_finish(const double *part, int PT, int batch, int64_t j0, int64_t count, int64_t steps,
                            double inv_n, double inv_gn, double *hist, void *stream);
int launch_zero(double *dst, int64_t count, void *stream);
int launch_col_multi(int prec, const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks,
                     int off, int64_t g, size_t lds, void *stream);
int launch_row_multi(int prec, const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks,
                     int off, int64_t g, size_t lds, void *stream);
// register-staged interior merge pass of the adjoint sweep; -1 when it does not apply
int launch_col_fast_adjoint(int prec, int variant, const ColArgs &a, int batch, void *stream);
// register-staged multi-member passes (kernels_fast.hip); -1 when the length
// has no such pass
// (variant 1: 256 threads x 16 elements, 2: 512 threads x 8; both on the
// members' 4096-element tiles)
// (columns: mid 0 the interior passes, 9 the members' first passes, 10 the
// last passes of the members whose schedules end at g)
int launch_col_fast_multi(int prec, int variant, int L1, int mid, const BatchDesc *d, const int *idx,
                          const int *start, int nmem, int nblocks, int off, int64_t g, void *stream);
int launch_row_fast_multi(int prec, int variant, int L2, int mid, const BatchDesc *d, const int *idx,
                          const int *start, int nmem, int nblocks, int off, int64_t g, void *stream);
int launch_resident_multi(int prec, const ResArgs *d, int ninst, size_t lds, void *stream);
int launch_ktab_multi(const KtabDesc *d, int count, int64_t max_len, void *stream);
int launch_permute_c128(void *dst, const void *src_nat, int64_t L, int L1, int L2, int transposed,
                        double scale, void *stream);
int launch_unpermute_c128(void *dst_nat, const void *src, int64_t L, int L1, int L2,
                          void *stream);
int launch_chirp_filter(void *dst_c128, int64_t N, int64_t L, void *stream);
int launch_reduce_batch(double *dst, const double *src, int64_t N, int batch, void *stream);
// dst[b][c][r] = src[b][r][c]: batch rows x cols matrices of 8- or 16-byte elements
int launch_transpose(int esize, void *dst, const void *src, int batch, int rows, int cols, int64_t dst_bs,
                     int64_t src_bs, void *stream);
int launch_ktab(double *dst, int64_t count, double kin, double scale, void *stream);
int diag_partials();  // blocks per state of launch_sums
int launch_sums(int prec, const void *x, int64_t x_bs, int64_t count, int batch, const int32_t *w,
                const double *vw, int64_t vw_bs, double *partial, void *stream);
int launch_col_inner(int prec, const ColArgs &a, int batch, void *stream);
int launch_proj_sums(int prec, const void *x, int64_t x_bs, int64_t count, int batch, double scale, int transposed,
                     int L1, int L2, const double *ghat, int64_t g_bs, double *partial, double *out, void *stream);
int launch_diag_finish(const double *pp, const double *ps, int batch, int64_t N, double gamma, double kscale,
                       double *out, void *stream);
int launch_conv_input(void *dst, const int32_t *s, const double *ktab, int64_t N, void *stream);
int launch_conv_embed(void *g, const void *src, int64_t N, int64_t L, double scale, void *stream);
int launch_spectrum_f32(void *dst, const void *src, int64_t count, void *stream);
int launch_phase_table(int prec, void *dst, const double *v, int64_t v_bs, int nv, int64_t N, double phase,
                       void *stream);
// fast register-staged variants (kernels_fast.hip); return -1 when the variant does not fit
int launch_col_fast(int prec, int variant, const ColArgs &a, int batch, void *stream);
int launch_row_fast(int prec, int variant, const RowArgs &a, int batch, void *stream);
bool fast_col_fits(int prec, int variant, int L1, int L2, int C);
bool fast_row_fits(int prec, int variant, int L1, int L2, int rows);
int kernels_init();  // raise dynamic LDS limits once

// Timing of one launch when timing is enabled (timing.cpp): a start / stop
// event pair registered under a kernel class, to be passed to
// hipExtLaunchKernelGGL so that the dispatch itself stamps them.  Both are
// null when timing is off.
void timing_events(int kind, void **start, void **stop);

}  // namespace lt

// ---------------------------------------------------------------- the plan
struct lt_plan {
    int d = 0, r = 0;
    int64_t n[4] = {1, 1, 1, 1};
    int64_t N = 0;
    std::vector<int64_t> Z;        // r x d
    std::vector<int32_t> H;        // user index set, nh x d
    std::vector<int64_t> key_of_h; // nh
    std::vector<int64_t> s_of_key; // N
    std::vector<int32_t> h_of_key; // N x d
    int64_t n_index = 0, n_completed = 0, max_s = 0;
    bool complete = true;          // give keys the index set leaves unowned their minimal-l2 representative
    // [0]: the run schedule; [1]: a two-pass schedule (used by the adjoint,
    // identical to [0] when [0] is already two-pass); [2]: the transposed
    // schedule of a rank-2 tensor whose columns are long (ok only then; runs
    // without checkpoints take it); inner index lt_prec
    lt::Sched sched[3][3];
    std::mutex mu;
    lt::DevTables dev[3][3];
    int device = -1;
};

namespace lt {
void set_error(const std::string &msg);
lt_status fail(lt_status st, const std::string &msg);
Sched make_schedule(const lt_plan &p, int prec, bool force_two_pass);
lt_status plan_index_set(lt_plan &p);
lt_status ensure_device_tables(lt_plan &p, int which, int prec, void *stream);
lt_status prepare_forward_tables(lt_plan &p, int prec, void *stream);
bool forward_tables_ready(lt_plan &p, int prec);
bool factor_radices(int64_t L, Radices &out, int max_log2 = 4);
int64_t smooth7_at_least(int64_t x);
}  // namespace lt
