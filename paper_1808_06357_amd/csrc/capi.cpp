// C-ABI of the lattice Strang library: argument checks, device tables and the
// launch sequences of a run (eq. (StrangTDSE) / Algorithm 1), its adjoint and
// batches of unrelated problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "lt_internal.h"

using namespace lt;

namespace {

constexpr long double kPiL = 3.141592653589793238462643383279502884L;

size_t esz(int prec) { return prec == LT_C128 ? 16 : 8; }

#define HIP_TRY(expr, what)                                                                    \
    do {                                                                                       \
        hipError_t e_ = (hipError_t)(expr);                                                    \
        if (e_ != hipSuccess)                                                                  \
            return fail(LT_E_HIP, std::string(what) + ": " + hipGetErrorString(e_));           \
    } while (0)

// exp(-2 pi i q mult / L) for q < count, computed in long double from the
// exactly reduced integer q*mult mod L.  complex128 tables: (re, im) doubles;
// complex64 tables: (hi.re, hi.im, lo.re, lo.im) floats with hi = fl(w) and
// lo = fl(w - hi), so that products can carry the table value beyond FP32.
std::vector<double> roots_d(int64_t L, int64_t count, int64_t mult)
{
    std::vector<double> out((size_t)(2 * count));
    for (int64_t q = 0; q < count; ++q) {
        const int64_t m = (int64_t)(((__int128)q * mult) % L);
        const long double a = 2.0L * kPiL * (long double)m / (long double)L;
        out[(size_t)(2 * q)] = (double)cosl(a);
        out[(size_t)(2 * q + 1)] = (double)(-sinl(a));
    }
    return out;
}

std::vector<float> roots_f(int64_t L, int64_t count, int64_t mult = 1)
{
    std::vector<float> out((size_t)(4 * count));
    for (int64_t q = 0; q < count; ++q) {
        const int64_t m = (int64_t)(((__int128)q * mult) % L);
        const long double a = 2.0L * kPiL * (long double)m / (long double)L;
        const long double c = cosl(a), s = -sinl(a);
        const float ch = (float)c, sh = (float)s;
        out[(size_t)(4 * q)] = ch;
        out[(size_t)(4 * q + 1)] = sh;
        out[(size_t)(4 * q + 2)] = (float)(c - (long double)ch);
        out[(size_t)(4 * q + 3)] = (float)(s - (long double)sh);
    }
    return out;
}

template <typename T>
lt_status upload(void **dst, const std::vector<T> &src, const char *what)
{
    HIP_TRY(hipMalloc(dst, std::max<size_t>(src.size() * sizeof(T), 16)), what);
    HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return LT_OK;
}

lt_status bind_device(lt_plan &p)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (p.device < 0) p.device = dev;
    if (p.device != dev) return fail(LT_E_ARG, "plan was first used on another device");
    kernels_init();
    return LT_OK;
}

bool transposed_layout(const Sched &s) { return s.passes == 2 && !s.rank2; }

// A two-pass rank-2 tensor n1 x n2 (row-major, n2 contiguous) whose columns
// of n1 points fill a tile with one or two columns, so that every element of a
// column pass sits on its own cache line: the same transform held transposed
// (n2 x n1) reads n2-point columns many to a tile and n1-point rows.  Not ok
// (unused) for other schedules.
Sched swapped_schedule(const Sched &s0)
{
    Sched s;
    if (!s0.ok || !s0.rank2 || s0.passes != 2 || s0.L1 < 2048 || (int64_t)s0.L2 * 4 > s0.L1) return s;
    s = s0;
    s.swapped = true;
    s.L1 = s0.L2;
    s.L2 = s0.L1;
    s.ra = s0.rb;
    s.rb = s0.ra;
    s.cols = (int)std::max<int64_t>(1, std::min<int64_t>(kTileElems / s.L1, s.L2));
    s.rows = (int)std::max<int64_t>(1, std::min<int64_t>(kTileElems / s.L2, s.L1));
    return s;
}

lt_status build_twiddles(lt_plan &p, int which, int prec)
{
    DevTables &D = p.dev[which][prec];
    const Sched &s = p.sched[which][prec];
    if (D.twa) return LT_OK;
    int64_t La, Lb;
    if (s.passes == 1) {
        La = s.rank2 ? s.L1 : s.L;
        Lb = s.rank2 ? s.L2 : 1;
    } else if (s.passes == 3) {
        La = s.L1;
        Lb = s.L3;  // the row pass
    } else {
        La = s.L1;
        Lb = s.L2;
    }
    lt_status st;
    if (prec == LT_C128) {
        if ((st = upload(&D.twa, roots_d(La, La, 1), "twiddles"))) return st;
        if ((st = upload(&D.twb, roots_d(Lb, Lb, 1), "twiddles"))) return st;
    } else {
        if ((st = upload(&D.twa, roots_f(La, La), "twiddles"))) return st;
        if ((st = upload(&D.twb, roots_f(Lb, Lb), "twiddles"))) return st;
    }
    if (transposed_layout(s)) {
        if ((st = upload((void **)&D.tw4hi, roots_d(s.L, s.L1, s.L2), "twiddles"))) return st;
        if ((st = upload((void **)&D.tw4lo, roots_d(s.L, s.L2, 1), "twiddles"))) return st;
    }
    if (s.passes == 3) {
        // outer four-step over L1 x M (M = L2 L3), inner four-step over L2 x L3
        const int64_t M = (int64_t)s.L2 * s.L3;
        if ((st = upload((void **)&D.tw4hi, roots_d(s.L, s.L1, M), "twiddles"))) return st;
        if ((st = upload((void **)&D.tw4lo, roots_d(s.L, M, 1), "twiddles"))) return st;
        if ((st = upload((void **)&D.tw4hi2, roots_d(M, s.L2, s.L3), "twiddles"))) return st;
        if ((st = upload((void **)&D.tw4lo2, roots_d(M, s.L3, 1), "twiddles"))) return st;
        if (prec == LT_C128) st = upload(&D.twc, roots_d(s.L2, s.L2, 1), "twiddles");
        else st = upload(&D.twc, roots_f(s.L2, s.L2), "twiddles");
        if (st) return st;
    }
    std::vector<int32_t> sk((size_t)p.N);
    for (int64_t t = 0; t < p.N; ++t) sk[(size_t)t] = (int32_t)p.s_of_key[(size_t)t];
    if ((st = upload((void **)&D.s_key, sk, "key norms"))) return st;
    if (s.passes >= 2 && !s.bluestein) {
        // kinetic angles are read at the row-pass positions
        std::vector<int32_t> sr((size_t)p.N);
        for (int64_t pos = 0; pos < p.N; ++pos) {
            int64_t chi = pos;
            if (transposed_layout(s) || s.swapped) {
                // rank-1 four-step: pos = k1 L2 + k2 holds xi = k1 + L1 k2; a
                // swapped rank-2 tensor: pos = k2 n1 + k1 holds (k1, k2), key
                // k1 n2 + k2 -- the same map with L1 = n2, L2 = n1
                const int64_t k1 = pos / s.L2, k2 = pos - k1 * s.L2;
                chi = k1 + (int64_t)s.L1 * k2;
            } else if (s.passes == 3) {
                // pos = k1 M + k2 L3 + k3 holds xi = k1 + L1 (k2 + L2 k3)
                const int64_t M = (int64_t)s.L2 * s.L3;
                const int64_t k1 = pos / M, rem = pos - k1 * M;
                const int64_t k2 = rem / s.L3, k3 = rem - k2 * s.L3;
                chi = k1 + (int64_t)s.L1 * (k2 + (int64_t)s.L2 * k3);
            }
            sr[(size_t)pos] = sk[(size_t)chi];
        }
        if ((st = upload((void **)&D.s_row, sr, "key norms"))) return st;
    }
    return LT_OK;
}

ColArgs col_base(const Sched &s, const DevTables &D, int64_t N)
{
    ColArgs a;
    std::memset(&a, 0, sizeof(a));
    a.L1 = s.L1;
    a.L2 = s.L2;
    a.C = s.cols;
    a.ntiles = (s.L2 + s.cols - 1) / s.cols;
    a.Nvalid = N;
    a.twiddle = s.rank2 ? 0 : 1;
    a.tw4hi = D.tw4hi;
    a.tw4lo = D.tw4lo;
    a.twa = D.twa;
    a.rad = s.ra;
    a.scale = 1.0;
    a.Nchirp = N;
    return a;
}

RowArgs row_base(const Sched &s, const DevTables &D)
{
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.L1 = s.L1;
    a.L2 = s.L2;
    a.rows = s.rows;
    a.nblk = (s.L1 + s.rows - 1) / s.rows;
    a.twb = D.twb;
    a.rad = s.rb;
    a.ktab_n = D.ktab_n;
    return a;
}

// kernel spectrum of the chirp-z convolution, natural order, complex double
lt_status bhat_natural(lt_plan &p, int which, void *nat, void *tmp, hipStream_t st)
{
    // built with the double-precision schedule of the same slot (same length
    // and layout as the run precision's)
    const Sched &s = p.sched[which][LT_C128];
    if (!s.ok) return fail(LT_E_UNSUPPORTED, "no double-precision schedule for the chirp-z kernel");
    lt_status r = build_twiddles(p, which, LT_C128);
    if (r) return r;
    const DevTables &D = p.dev[which][LT_C128];
    HIP_TRY(launch_chirp_filter(tmp, p.N, s.L, st), "chirp filter");
    if (s.passes == 1) {
        HIP_TRY(launch_fft_single(s.ra, D.twa, tmp, s.L, st), "kernel spectrum");
        HIP_TRY(hipMemcpyAsync(nat, tmp, (size_t)s.L * 16, hipMemcpyDeviceToDevice, st), "copy");
        return LT_OK;
    }
    ColArgs c = col_base(s, D, s.L);
    c.buf = tmp;
    c.post_fwd = 1;
    HIP_TRY(launch_col(LT_C128, s, c, 1, st), "kernel spectrum (columns)");
    RowArgs rw = row_base(s, D);
    rw.buf = tmp;
    rw.fft_only = 1;
    HIP_TRY(launch_row(LT_C128, s, rw, 1, st), "kernel spectrum (rows)");
    HIP_TRY(launch_unpermute_c128(nat, tmp, s.L, s.L1, s.L2, st), "kernel spectrum (order)");
    return LT_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// forward runs: the kinetic table (one complex double per squared norm
// 0..max_s), for two-pass chirp-z a transform buffer (otherwise the transform
// runs in u itself), and for two-pass runs the merged potential multiplier
// exp(-i dt v / gamma) per point (one table per distinct potential)
struct RunWork {
    size_t ktab = 0, w = 0, ptab = 0, conv = 0, conv_tmp = 0, conv_f = 0, total = 0;
};

RunWork run_layout(const lt_plan &p, const Sched &s, int prec, int batch, bool shared_v = true,
                   bool phase_table = true, bool conv_space = true)
{
    RunWork w;
    w.ktab = 0;
    size_t off = align_up((size_t)(p.max_s + 1) * 16);
    w.w = off;
    if (s.bluestein && s.passes == 2) off = align_up(off + (size_t)batch * s.L * esz(prec));
    w.ptab = off;
    if (s.passes >= 2 && phase_table)
        off = align_up(off + (size_t)(shared_v ? 1 : batch) * p.N * 16);
    if (s.bluestein && s.passes == 2 && conv_space) {
        // kernel spectrum of the step's cyclic convolution (complex double, L)
        // and a complex-double scratch vector of N
        w.conv = off;
        off = align_up(off + (size_t)s.L * 16);
        w.conv_tmp = off;
        off = align_up(off + (size_t)p.N * 16);
        if (prec == LT_C64) {  // the spectrum rounded to complex float for the complex64 rows
            w.conv_f = off;
            off = align_up(off + (size_t)s.L * 8);
        }
    }
    w.total = off;
    return w;
}

struct AdjWork {
    size_t ktab = 0, w = 0, gacc = 0, ptab = 0, conv = 0, conv_tmp = 0, conv_f = 0, ut = 0, gt = 0, vt = 0,
           total = 0;
};

// The adjoint sweep's schedule slot: the swapped one of a rank-2 tensor with
// long columns (the sweep then runs transposed, like the forward run), else
// slot 1.
int adj_slot(const lt_plan &p, int prec) { return p.sched[2][prec].ok ? 2 : 1; }

AdjWork adj_layout(const lt_plan &p, const Sched &s, int prec, int batch, bool shared_v)
{
    AdjWork w;
    size_t off = align_up((size_t)(p.max_s + 1) * 16);
    w.w = off;
    off = align_up(off + (size_t)2 * batch * s.L * esz(prec));   // state and cotangent
    w.gacc = off;
    off = align_up(off + (size_t)batch * p.N * sizeof(double));
    w.ptab = off;  // the interior merge passes' potential phase per point
    off = align_up(off + (size_t)(shared_v ? 1 : batch) * p.N * 16);
    if (s.bluestein) {  // the convolution form's spectrum and scratch
        w.conv = off;
        off = align_up(off + (size_t)s.L * 16);
        w.conv_tmp = off;
        off = align_up(off + (size_t)p.N * 16);
        if (prec == LT_C64) {  // the spectrum rounded to complex float for the complex64 rows
            w.conv_f = off;
            off = align_up(off + (size_t)s.L * 8);
        }
    }
    if (s.swapped) {
        // transposed u(T) (later dJ/du0), transposed cotangent (later the
        // shared gradient), transposed v
        w.ut = off;
        off = align_up(off + (size_t)batch * p.N * esz(prec));
        w.gt = off;
        off = align_up(off + (size_t)batch * p.N * esz(prec));
        w.vt = off;
        off = align_up(off + (size_t)(shared_v ? 1 : batch) * p.N * sizeof(double));
    }
    w.total = off;
    return w;
}

bool finite(double x) { return std::isfinite(x); }

lt_status check_common(const lt_plan *p, lt_prec prec, int32_t batch, double gamma, double dt,
                       int64_t steps)
{
    if (!p) return fail(LT_E_ARG, "plan is NULL");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "prec must be LT_C64 or LT_C128");
    if (batch < 0) return fail(LT_E_ARG, "batch must be >= 0");
    if (!(gamma > 0) || !finite(gamma)) return fail(LT_E_ARG, "gamma must be finite and > 0");
    if (!finite(dt)) return fail(LT_E_ARG, "dt must be finite");
    if (steps < 0) return fail(LT_E_ARG, "steps must be >= 0");
    if (!p->sched[0][prec].ok)
        return fail(LT_E_UNSUPPORTED, "no GPU schedule for this lattice in this precision");
    return LT_OK;
}

struct Scratch {
    void *ptr = nullptr;
    hipStream_t st = nullptr;
    bool owned = false;
    ~Scratch()
    {
        if (owned && ptr) hipFreeAsync(ptr, st);
    }
};

lt_status get_work(Scratch &sc, void *work, size_t work_bytes, size_t need, hipStream_t st)
{
    sc.st = st;
    if (need == 0) return LT_OK;
    if (work) {
        if (work_bytes < need)
            return fail(LT_E_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
        sc.ptr = work;
        return LT_OK;
    }
    HIP_TRY(hipMallocAsync(&sc.ptr, need, st), "workspace allocation");
    sc.owned = true;
    return LT_OK;
}

inline char *at(void *base, size_t off) { return (char *)base + off; }

double kinetic_angle(double gamma, double dt) { return 2.0 * M_PI * M_PI * gamma * dt; }

// exp(-i 2 pi^2 gamma dt m) * scale for every squared norm m of the plan
lt_status make_ktab(const lt_plan &p, const Sched &s, double *ktab, double gamma, double dt, hipStream_t st)
{
    const double scale = s.bluestein ? 1.0 : 1.0 / (double)s.L;
    HIP_TRY(launch_ktab(ktab, p.max_s + 1, kinetic_angle(gamma, dt), scale, st), "kinetic table");
    return LT_OK;
}

// launch arguments of the two-pass sequence, per role: the first column pass
// (half potential step, chirp), the merged potential step P^2 between steps,
// the chirp-z kinetic column pass, the last column pass, and the row pass
struct Roles {
    ColArgs first, pot, kin, last;
    RowArgs row;
};

Roles two_pass_roles(const Sched &s, const DevTables &D, int64_t N, const double *v, int64_t v_stride, void *u,
                     void *W, double half, const double *ktab, const void *ptab = nullptr)
{
    Roles R;
    void *buf = s.bluestein ? W : u;
    const int64_t buf_bs = s.bluestein ? s.L : N;
    R.first = col_base(s, D, N);
    R.first.buf = buf;
    R.first.buf_bs = buf_bs;
    R.first.in = u;
    R.first.in_bs = N;
    R.first.post_fwd = 1;
    R.first.v = v;
    R.first.v_bs = v_stride;
    R.first.phase = half;
    R.first.chirp = s.bluestein ? 1 : 0;
    R.row = row_base(s, D);
    R.row.buf = buf;
    R.row.buf_bs = buf_bs;
    if (s.bluestein) {
        R.row.bhat = D.bhat;
    } else {
        R.row.s = D.s_row;
        R.row.ktab = ktab;
    }
    ColArgs mid = col_base(s, D, N);
    mid.buf = buf;
    mid.buf_bs = buf_bs;
    mid.pre_inv = 1;
    mid.post_fwd = 1;
    R.kin = mid;  // chirp-z: kinetic phase at the natural spectral index
    R.kin.s = D.s_key;
    R.kin.ktab = ktab;
    R.pot = mid;
    R.pot.v = v;
    R.pot.v_bs = v_stride;
    R.pot.phase = 2.0 * half;
    R.pot.ptab = ptab;
    R.pot.ptab_bs = v_stride ? N : 0;
    R.last = col_base(s, D, N);
    R.last.buf = buf;
    R.last.buf_bs = buf_bs;
    R.last.pre_inv = 1;
    R.last.out = u;
    R.last.out_bs = N;
    R.last.v = v;
    R.last.v_bs = v_stride;
    R.last.phase = half;
    R.last.chirp = s.bluestein ? -1 : 0;
    return R;
}

// Chirp-z lattices: the kinetic part F^-1 K F of a step is the cyclic
// convolution of length N with kernel k = conj(F conj(K)) / sqrt(N), i.e.
// k_j = (1/N) sum_xi K_xi exp(2 pi i xi j / N).  Embedded with zero padding in
// the length L >= 2N-1 of the chirp-z schedule (g_j = k_j, g_{L-j} = k_{N-j}),
// it becomes one length-L FFT pair, so a step needs two passes instead of the
// four of a chirp-z DFT and its inverse.  This builds the spectrum
// G = FFT_L(g) / L in complex double, in the row pass layout: k from one
// chirp-z DFT of conj(K), then the embedding and one forward FFT.
lt_status conv_spectrum(lt_plan &p, int which, const double *ktab, void *G, void *tmp, hipStream_t st)
{
    const Sched &s = p.sched[which][LT_C128];
    const DevTables &D = p.dev[which][LT_C128];
    const int64_t N = p.N;
    HIP_TRY(launch_conv_input(tmp, D.s_key, ktab, N, st), "convolution kernel");
    ColArgs a = col_base(s, D, N);
    a.buf = G;
    a.buf_bs = s.L;
    a.in = tmp;
    a.in_bs = N;
    a.post_fwd = 1;
    a.chirp = 1;
    HIP_TRY(launch_col(LT_C128, s, a, 1, st), "convolution kernel");
    RowArgs r = row_base(s, D);
    r.buf = G;
    r.buf_bs = s.L;
    r.bhat = D.bhat;
    HIP_TRY(launch_row(LT_C128, s, r, 1, st), "convolution kernel");
    ColArgs c = col_base(s, D, N);
    c.buf = G;
    c.buf_bs = s.L;
    c.pre_inv = 1;
    c.out = tmp;
    c.out_bs = N;
    c.chirp = 1;
    HIP_TRY(launch_col(LT_C128, s, c, 1, st), "convolution kernel");  // tmp = F conj(K)
    HIP_TRY(launch_conv_embed(G, tmp, N, s.L, 1.0 / ((double)s.L * std::sqrt((double)N)), st),
            "convolution kernel");
    ColArgs f = col_base(s, D, s.L);
    f.buf = G;
    f.buf_bs = s.L;
    f.post_fwd = 1;
    HIP_TRY(launch_col(LT_C128, s, f, 1, st), "convolution kernel");
    RowArgs rf = row_base(s, D);
    rf.buf = G;
    rf.buf_bs = s.L;
    rf.fft_only = 1;
    HIP_TRY(launch_row(LT_C128, s, rf, 1, st), "convolution kernel");
    return LT_OK;
}

// runs at least this long use the convolution form on chirp-z lattices (its
// spectrum costs about five passes once)
constexpr int64_t kConvMinSteps = 4;

// the convolution form needs the complex128 schedule of the same slot with the
// same transform layout (its spectrum is built in double precision)
bool conv_available(const lt_plan &p, int which, const Sched &s)
{
    const Sched &d = p.sched[which][LT_C128];
    return s.bluestein && s.passes == 2 && d.ok && d.passes == 2 && d.L == s.L && d.L1 == s.L1 && d.L2 == s.L2;
}

// Per-step sums of a run (Sec. 3.3 norm and potential energy at every step
// boundary j = 0..steps).  The passes at a boundary write per-tile partials
// into slot j mod CH of `part` ([slot][b][PT][2], PT bounding the tiles of
// any column launch of the schedule); every CH steps, and after the last, one
// launch reduces the filled slots into hist[b][j][2] in a fixed order and the
// slots are cleared for reuse.  The partial area is capped (kSumBytes).
constexpr size_t kSumBytes = size_t(64) << 20;

struct SumSink {
    double *part = nullptr, *hist = nullptr;
    int PT = 1, batch = 1;
    int64_t CH = 1, steps = 0, N = 1;
    double gamma = 1.0;
    explicit operator bool() const { return hist != nullptr; }
    double *slot(int64_t j) const { return part + (size_t)(j % CH) * batch * PT * 2; }
};

// tiles of the widest column launch of a schedule (row length L2, or L2 L3 for
// the outer pass of three levels): every kernel variant holds at least
// min(cols, 1024 / L1) columns per tile, and at least one
int sum_tiles(const Sched &s)
{
    const int64_t M = s.passes == 3 ? (int64_t)s.L2 * s.L3 : (int64_t)s.L2;
    if (s.passes == 1) return 1;
    int c = std::max(1, std::min(s.cols, s.L1 <= 1024 ? 1024 / s.L1 : 1));
    return (int)((M + c - 1) / c);
}

int64_t sum_slots(int batch, int PT, int64_t steps, bool one_launch = false)
{
    if (one_launch) return steps + 1;  // a resident run writes every step from one launch
    const int64_t per = (int64_t)batch * PT * 16;
    return std::max<int64_t>(1, std::min<int64_t>(steps + 1, (int64_t)(kSumBytes / (size_t)std::max<int64_t>(per, 1))));
}

size_t sum_bytes(const Sched &s, int batch, int64_t steps)
{
    const int PT = sum_tiles(s);
    return align_up((size_t)sum_slots(batch, PT, steps, s.passes == 1) * batch * PT * 16);
}

SumSink make_sink(const Sched &s, int batch, int64_t steps, int64_t N, double gamma, void *part, double *hist)
{
    SumSink k;
    if (!hist) return k;
    k.part = (double *)part;
    k.hist = hist;
    k.PT = sum_tiles(s);
    k.batch = batch;
    k.steps = steps;
    k.N = N;
    k.gamma = gamma;
    k.CH = sum_slots(batch, k.PT, steps, s.passes == 1);
    return k;
}

lt_status sums_begin(const SumSink &k, hipStream_t st)
{
    if (!k) return LT_OK;
    HIP_TRY(launch_zero(k.part, k.CH * k.batch * k.PT * 2, st), "step sums");
    return LT_OK;
}

// after the pass that wrote boundary j: reduce a full chunk (or the last one)
lt_status sums_after(const SumSink &k, int64_t j, hipStream_t st)
{
    if (!k) return LT_OK;
    if ((j + 1) % k.CH != 0 && j != k.steps) return LT_OK;
    const int64_t j0 = j - j % k.CH;
    HIP_TRY(launch_step_sums_finish(k.part, k.PT, k.batch, j0, j - j0 + 1, k.steps, 1.0 / (double)k.N,
                                    1.0 / (k.gamma * (double)k.N), k.hist, st),
            "step sums");
    if (j != k.steps) HIP_TRY(launch_zero(k.part, k.CH * k.batch * k.PT * 2, st), "step sums");
    return LT_OK;
}

void sums_on(ColArgs &a, const SumSink &k, int64_t j, const double *v)
{
    if (!k) return;
    a.sum_part = k.slot(j);
    a.sum_pt = k.PT;
    a.sum_v = v;
}

// forward run of a state batch through the two-pass sequence; `conv` (chirp-z
// lattices) is the spectrum from conv_spectrum, or null for the chirp-z DFT
// pair per step.  A complex64 run given `conv_f` (L complex floats) rounds the
// spectrum into it once, and its register-staged rows read that copy: half
// the spectrum's bytes, applied in float (complex64 arithmetic, like the
// state); the general row kernel, where one runs, reads the double spectrum.
lt_status two_pass_forward(lt_plan &p, const Sched &s, const DevTables &D, int prec, int batch,
                           const double *v, int64_t v_stride, void *u, double gamma, double dt,
                           int64_t steps, void *ckpt, int64_t ck_every, const double *ktab, void *W,
                           void *ptab, const void *conv, hipStream_t st, bool ck_transposed = false,
                           const SumSink &sums = SumSink(), void *conv_f = nullptr)
{
    const int64_t N = p.N;
    const size_t S = esz(prec);
    const double half = dt / (2.0 * gamma);
    if (ptab && steps > 1)
        HIP_TRY(launch_phase_table(prec, ptab, v, v_stride, v_stride ? batch : 1, N, 2.0 * half, st),
                "potential table");
    Roles R = two_pass_roles(s, D, N, v, v_stride, u, W, half, ktab, ptab);
    const bool chirpz = s.bluestein && !conv;
    if (conv) {
        R.first.chirp = 0;
        R.last.chirp = 0;
        R.row.bhat = (const double *)conv;
        if (conv_f && prec == LT_C64) {
            HIP_TRY(launch_spectrum_f32(conv_f, conv, s.L, st), "convolution spectrum (complex float)");
            R.row.bhat_f = (const float *)conv_f;
        }
    }
    lt_status ls;
    if ((ls = sums_begin(sums, st))) return ls;
    sums_on(R.first, sums, 0, v);
    HIP_TRY(launch_col(prec, s, R.first, batch, st), "column pass");
    if ((ls = sums_after(sums, 0, st))) return ls;
    for (int64_t t = 0; t < steps; ++t) {
        R.row.conj_tab = 0;
        HIP_TRY(launch_row(prec, s, R.row, batch, st), "row pass");
        if (chirpz) {
            HIP_TRY(launch_col(prec, s, R.kin, batch, st), "column pass (kinetic)");
            R.row.conj_tab = 1;
            HIP_TRY(launch_row(prec, s, R.row, batch, st), "row pass");
        }
        if (t == steps - 1) break;
        ColArgs m = R.pot;
        const int64_t k = t + 1;  // state index at this merge point
        if (ckpt && k % ck_every == 0) {
            m.ck = at(ckpt, (size_t)(k / ck_every) * batch * N * S);
            m.ck_bs = N;
            m.ck_v = v;
            m.ck_phase = half;
            m.ck_chirp = chirpz ? 1 : 0;
            m.ck_t = ck_transposed ? 1 : 0;
        }
        sums_on(m, sums, k, v);
        HIP_TRY(launch_col(prec, s, m, batch, st), "column pass (potential)");
        if ((ls = sums_after(sums, k, st))) return ls;
    }
    sums_on(R.last, sums, steps, v);
    HIP_TRY(launch_col(prec, s, R.last, batch, st), "column pass (last)");
    return sums_after(sums, steps, st);
}

// Three-level run (power-of-two L of 2^24 points or more, L = L1 L2 L3, M =
// L2 L3): each step is the inner forward column pass over L2 inside each of
// the L1 blocks of M points, the row pass over L3 (kinetic step), the inner
// inverse column pass, then the outer column pass over L1 (row length M)
// with the merged potential step.  Spectrum index xi = k1 + L1 (k2 + L2 k3)
// sits at k1 M + k2 L3 + k3; the plan's row-order norms follow it.
lt_status three_level_forward(lt_plan &p, const Sched &s, const DevTables &D, int prec, int batch,
                              const double *v, int64_t v_stride, void *u, double gamma, double dt,
                              int64_t steps, void *ckpt, int64_t ck_every, const double *ktab, void *ptab,
                              hipStream_t st, const SumSink &sums = SumSink())
{
    const int64_t N = p.N, M = (int64_t)s.L2 * s.L3;
    const size_t S = esz(prec);
    const double half = dt / (2.0 * gamma);
    if (ptab && steps > 1)
        HIP_TRY(launch_phase_table(prec, ptab, v, v_stride, v_stride ? batch : 1, N, 2.0 * half, st),
                "potential table");
    ColArgs a;
    std::memset(&a, 0, sizeof(a));
    a.L1 = s.L1;
    a.L2 = (int)M;
    a.C = s.cols;
    a.ntiles = (int)(M / s.cols);
    a.Nvalid = N;
    a.twiddle = 1;
    a.tw4hi = D.tw4hi;
    a.tw4lo = D.tw4lo;
    a.twa = D.twa;
    a.rad = s.ra;
    a.scale = 1.0;
    a.buf = u;
    a.buf_bs = N;
    a.v = v;
    a.v_bs = v_stride;
    ColArgs first = a, pot = a, last = a;
    first.in = u;
    first.in_bs = N;
    first.post_fwd = 1;
    first.phase = half;
    pot.pre_inv = 1;
    pot.post_fwd = 1;
    pot.phase = 2.0 * half;
    pot.ptab = ptab;
    pot.ptab_bs = v_stride ? N : 0;
    last.pre_inv = 1;
    last.out = u;
    last.out_bs = N;
    last.phase = half;
    // the inner level: columns of L2 points, stride L3, in each block of M
    ColArgs in;
    std::memset(&in, 0, sizeof(in));
    in.L1 = s.L2;
    in.L2 = s.L3;
    in.C = s.cols2;
    in.ntiles = s.L3 / s.cols2;
    in.Nvalid = M;
    in.twiddle = 1;
    in.tw4hi = D.tw4hi2;
    in.tw4lo = D.tw4lo2;
    in.twa = D.twc;
    in.rad = s.rc;
    in.scale = 1.0;
    in.buf = u;
    in.buf_bs = M;
    ColArgs fwd = in, inv = in;
    fwd.post_fwd = 1;
    inv.pre_inv = 1;
    const int blocks = batch * s.L1;
    // rows of L3 points, L1 L2 of them per state
    RowArgs r;
    std::memset(&r, 0, sizeof(r));
    r.buf = u;
    r.buf_bs = N;
    r.L1 = s.L1 * s.L2;
    r.L2 = s.L3;
    r.rows = s.rows;
    r.nblk = r.L1 / r.rows;
    r.s = D.s_row;
    r.ktab = ktab;
    r.ktab_n = D.ktab_n;
    r.twb = D.twb;
    r.rad = s.rb;
    lt_status ls;
    if ((ls = sums_begin(sums, st))) return ls;
    sums_on(first, sums, 0, v);
    HIP_TRY(launch_col(prec, s, first, batch, st), "column pass");
    if ((ls = sums_after(sums, 0, st))) return ls;
    for (int64_t t = 0; t < steps; ++t) {
        HIP_TRY(launch_col_inner(prec, fwd, blocks, st), "inner column pass");
        HIP_TRY(launch_row(prec, s, r, batch, st), "row pass");
        HIP_TRY(launch_col_inner(prec, inv, blocks, st), "inner column pass");
        if (t == steps - 1) break;
        ColArgs m = pot;
        const int64_t k = t + 1;
        if (ckpt && k % ck_every == 0) {
            m.ck = at(ckpt, (size_t)(k / ck_every) * batch * N * S);
            m.ck_bs = N;
            m.ck_v = v;
            m.ck_phase = half;
        }
        sums_on(m, sums, k, v);
        HIP_TRY(launch_col(prec, s, m, batch, st), "column pass (potential)");
        if ((ls = sums_after(sums, k, st))) return ls;
    }
    sums_on(last, sums, steps, v);
    HIP_TRY(launch_col(prec, s, last, batch, st), "column pass (last)");
    return sums_after(sums, steps, st);
}

// ---------------------------------------------------------------- batches
// workspace of a batch: per problem its run workspace, then the descriptor
// block (kinetic-table, resident and two-pass descriptors, block prefix sums)
struct BatchLayout {
    std::vector<size_t> off;
    size_t desc = 0, d_ktab = 0, d_res = 0, d_two = 0, d_lists = 0, desc_bytes = 0, total = 0;
};

// kernel classes of a batch's pass launches: members listed by index into the
// descriptor array (longest schedules first, so the members still running at
// pass g are a prefix), with prefix sums of their blocks
constexpr int kMaxBatchLists = 32;  // general + register-staged classes, columns and rows

struct MemberList {
    int key = 0;                 // fast length (columns: L1; rows: 2 L2 + multiplier kind), -1 general
    std::vector<int> mem;        // member indices into the descriptor array
    std::vector<int> start;      // block prefix sums, size mem + 1
    std::vector<int64_t> npass;  // per member
    size_t idx_off = 0, start_off = 0;  // int offsets in the list area
    int act = 0;                 // members still running at the current pass
    int var = 1;                 // register-staged kernel geometry (1: 256 x 16, 2: 512 x 8, 5: 256 x 8
                                 // on 2048-element tiles)
};

BatchLayout batch_layout(int32_t B, const lt_plan *const *plans, int prec)
{
    BatchLayout b;
    size_t off = 0;
    b.off.resize(B);
    for (int i = 0; i < B; ++i) {
        b.off[i] = off;
        off += run_layout(*plans[i], plans[i]->sched[0][prec], prec, 1, true, true, true).total;
    }
    b.desc = off;
    size_t d = 0;
    b.d_ktab = d;
    d = align_up(d + (size_t)B * sizeof(KtabDesc));
    b.d_res = d;
    d = align_up(d + (size_t)B * sizeof(ResArgs));
    b.d_two = d;
    d = align_up(d + (size_t)B * sizeof(BatchDesc));
    b.d_lists = d;  // each member once in a column list and once in a row list
    d = align_up(d + (size_t)(4 * B + 2 * kMaxBatchLists) * sizeof(int));
    b.desc_bytes = d;
    b.total = off + d;
    return b;
}

// pinned staging buffer for descriptor uploads; the event of the last copy
// guards its reuse
struct Staging {
    std::mutex mu;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
Staging g_stage;

lt_status upload_async(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_stage.mu);
    if (g_stage.done) HIP_TRY(hipEventSynchronize(g_stage.done), "staging wait");
    if (bytes > g_stage.cap) {
        if (g_stage.host) HIP_TRY(hipHostFree(g_stage.host), "staging free");
        g_stage.host = nullptr;
        g_stage.cap = 0;
        HIP_TRY(hipHostMalloc(&g_stage.host, bytes, hipHostMallocDefault), "staging allocation");
        g_stage.cap = bytes;
    }
    if (!g_stage.done) HIP_TRY(hipEventCreateWithFlags(&g_stage.done, hipEventDisableTiming), "event");
    std::memcpy(g_stage.host, src, bytes);
    HIP_TRY(hipMemcpyAsync(dst, g_stage.host, bytes, hipMemcpyHostToDevice, st), "descriptor upload");
    HIP_TRY(hipEventRecord(g_stage.done, st), "event record");
    return LT_OK;
}

// a second stream per device (default priority) for work that overlaps the
// caller's stream
lt_status side_stream(hipStream_t *out)
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "device query");
    if (dev < 0 || dev >= 64) return fail(LT_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[dev]) HIP_TRY(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking), "stream");
    *out = streams[dev];
    return LT_OK;
}

}  // namespace

// ---------------------------------------------------------------- device tables
namespace lt {
lt_status ensure_device_tables(lt_plan &p, int which, int prec, void *stream)
{
    std::lock_guard<std::mutex> lock(p.mu);
    DevTables &D = p.dev[which][prec];
    if (D.built) return LT_OK;
    D.ktab_n = p.max_s + 1;
    const Sched &s = p.sched[which][prec];
    if (!s.ok) return fail(LT_E_UNSUPPORTED, "no GPU schedule for this lattice in this precision");
    lt_status r = bind_device(p);
    if (r) return r;
    if ((r = build_twiddles(p, which, prec))) return r;
    hipStream_t st = (hipStream_t)stream;
    if (s.bluestein) {
        void *nat = nullptr, *tmp = nullptr;
        HIP_TRY(hipMalloc(&nat, (size_t)s.L * 16), "chirp-z tables");
        HIP_TRY(hipMalloc(&tmp, (size_t)s.L * 16), "chirp-z tables");
        HIP_TRY(hipMalloc((void **)&D.bhat, (size_t)s.L * 16), "chirp-z tables");
        r = bhat_natural(p, which, nat, tmp, st);
        if (!r) {
            const double scale = 1.0 / ((double)s.L * std::sqrt((double)p.N));
            hipError_t e = (hipError_t)launch_permute_c128(D.bhat, nat, s.L, s.L1, s.L2,
                                                           transposed_layout(s) ? 1 : 0, scale, st);
            if (e != hipSuccess) r = fail(LT_E_HIP, std::string("kernel spectrum: ") + hipGetErrorString(e));
        }
        hipError_t e = hipStreamSynchronize(st);
        hipFree(nat);
        hipFree(tmp);
        if (r) return r;
        if (e != hipSuccess) return fail(LT_E_HIP, std::string("table build: ") + hipGetErrorString(e));
    }
    D.built = true;
    return LT_OK;
}

// Whether the device tables a forward run in precision prec reads exist
// (then a run with a caller workspace allocates nothing).
bool forward_tables_ready(lt_plan &p, int prec)
{
    std::lock_guard<std::mutex> lock(p.mu);
    const int which = p.sched[2][prec].ok ? 2 : 0;
    if (!p.dev[which][prec].built) return false;
    const Sched &s = p.sched[which][prec];
    if (s.bluestein && s.passes == 2 && p.sched[0][LT_C128].ok) return p.dev[0][LT_C128].built;
    return true;
}

// Device tables a forward run in precision prec reads: its schedule's (the
// swapped one for a rank-2 tensor with long columns), plus the complex128
// tables of a two-pass chirp-z lattice, whose convolution spectrum is built
// in double precision.
lt_status prepare_forward_tables(lt_plan &p, int prec, void *stream)
{
    const int which = p.sched[2][prec].ok ? 2 : 0;
    lt_status st = ensure_device_tables(p, which, prec, stream);
    if (st) return st;
    const Sched &s = p.sched[which][prec];
    if (s.bluestein && s.passes == 2 && p.sched[0][LT_C128].ok) return ensure_device_tables(p, 0, LT_C128, stream);
    return LT_OK;
}

// Workspace of a run on the swapped rank-2 schedule: the run's own layout,
// then the transposed state (batch x N) and potential (1 or batch x N).
struct SwapWork {
    RunWork run;
    size_t u = 0, v = 0, total = 0;
};

SwapWork swap_layout(const lt_plan &p, const Sched &s, int prec, int batch, bool shared_v)
{
    SwapWork w;
    w.run = run_layout(p, s, prec, batch, shared_v);
    size_t off = w.run.total;
    w.u = off;
    off = align_up(off + (size_t)batch * p.N * esz(prec));
    w.v = off;
    off = align_up(off + (size_t)(shared_v ? 1 : batch) * p.N * sizeof(double));
    w.total = off;
    return w;
}

// A run of a rank-2 tensor on its swapped schedule: the state and the
// potential are transposed into the workspace (n2 x n1), the steps run there
// (checkpoints are stored in lattice order by the checkpoint passes), and the
// state is transposed back.
lt_status swapped_forward(lt_plan &p, int prec, int batch, const double *v, int64_t v_stride, void *u,
                          double gamma, double dt, int64_t steps, void *ckpt, int64_t ckpt_every, double *sums,
                          void *work, size_t work_bytes, void *stream)
{
    hipStream_t hs = (hipStream_t)stream;
    lt_status st;
    if ((st = ensure_device_tables(p, 2, prec, stream))) return st;
    const Sched &s = p.sched[2][prec];
    const DevTables &D = p.dev[2][prec];
    const bool shared = v_stride == 0;
    const SwapWork L = swap_layout(p, s, prec, batch, shared);
    const size_t need = L.total + (sums ? sum_bytes(s, batch, steps) : 0);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, need, hs))) return st;
    const SumSink sink = make_sink(s, batch, steps, p.N, gamma, at(sc.ptr, L.total), sums);
    double *ktab = (double *)at(sc.ptr, L.run.ktab);
    if ((st = make_ktab(p, s, ktab, gamma, dt, hs))) return st;
    const int n1 = s.L2, n2 = s.L1;
    void *U = at(sc.ptr, L.u);
    double *V = (double *)at(sc.ptr, L.v);
    if (ckpt)
        HIP_TRY(hipMemcpyAsync(ckpt, u, (size_t)batch * p.N * esz(prec), hipMemcpyDeviceToDevice, hs),
                "checkpoint 0");
    HIP_TRY(launch_transpose((int)esz(prec), U, u, batch, n1, n2, p.N, p.N, hs), "state transpose");
    HIP_TRY(launch_transpose(8, V, v, shared ? 1 : batch, n1, n2, p.N, shared ? p.N : v_stride, hs),
            "potential transpose");
    if ((st = two_pass_forward(p, s, D, prec, batch, V, shared ? 0 : p.N, U, gamma, dt, steps, ckpt,
                               ckpt ? ckpt_every : 0, ktab, at(sc.ptr, L.run.w), at(sc.ptr, L.run.ptab), nullptr,
                               hs, true, sink)))
        return st;
    HIP_TRY(launch_transpose((int)esz(prec), u, U, batch, n2, n1, p.N, p.N, hs), "state transpose");
    return LT_OK;
}
}  // namespace lt

// ---------------------------------------------------------------- C-ABI
extern "C" {

lt_status lattice_plan(int32_t d, int32_t r, const int64_t *Z, const int64_t *n, const int32_t *H,
                       int64_t nh, int32_t complete, int32_t prec_mask, lt_plan **out)
{
    if (!out) return fail(LT_E_ARG, "out is NULL");
    *out = nullptr;
    if (complete != 0 && complete != 1) return fail(LT_E_ARG, "complete must be 0 or 1");
    if (prec_mask & ~(LT_C64 | LT_C128)) return fail(LT_E_ARG, "prec_mask must combine LT_C64 and LT_C128");
    if (d < 1 || d > 64) return fail(LT_E_ARG, "d must be in [1, 64]");
    if (r < 1 || r > 4) return fail(LT_E_ARG, "r must be in [1, 4]");
    if (!Z || !n) return fail(LT_E_ARG, "Z and n must not be NULL");
    if (nh < 0 || (nh > 0 && !H)) return fail(LT_E_ARG, "H must hold nh >= 0 rows");
    __int128 N = 1;
    for (int i = 0; i < r; ++i) {
        if (n[i] < 1) return fail(LT_E_ARG, "moduli must be >= 1");
        if (i > 0 && n[i - 1] % n[i] != 0)
            return fail(LT_E_NOT_CANONICAL, "moduli must satisfy n_{i+1} | n_i (Def. 1)");
        N *= n[i];
        if (N > ((__int128)1 << 31) - 1) return fail(LT_E_UNSUPPORTED, "N must be below 2^31");
    }
    for (int64_t t = 0; t < nh * d; ++t)
        if (H[t] < -(1 << 24) || H[t] > (1 << 24)) return fail(LT_E_ARG, "index set entries too large");
    lt_plan *p = new (std::nothrow) lt_plan;
    if (!p) return fail(LT_E_NOMEM, "plan allocation");
    p->d = d;
    p->r = r;
    for (int i = 0; i < r; ++i) p->n[i] = n[i];
    p->N = (int64_t)N;
    p->complete = complete != 0;
    try {
        p->Z.assign(Z, Z + (size_t)r * d);
        if (H) p->H.assign(H, H + (size_t)nh * d);
        lt_status st = plan_index_set(*p);
        if (st != LT_OK) {
            delete p;
            return st;
        }
        for (int prec : {LT_C64, LT_C128}) {
            p->sched[0][prec] = make_schedule(*p, prec, false);
            p->sched[1][prec] = p->sched[0][prec].passes == 2 ? p->sched[0][prec]
                                                              : make_schedule(*p, prec, true);
            p->sched[2][prec] = swapped_schedule(p->sched[0][prec]);
        }
        // complex128 column passes default to the 256 x 8 geometry on
        // 2048-element tiles where it fits: with the step's fused sums the
        // 16-element geometries run out of registers and spill
        for (int w = 0; w < 3; ++w) {
            Sched &s = p->sched[w][LT_C128];
            if (s.ok && s.passes == 2 && fast_col_fits(LT_C128, 5, s.L1, s.L2, s.cols)) s.col_var = s.col_var_m = 5;
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(LT_E_NOMEM, "out of host memory while planning");
    }
    for (int prec : {LT_C64, LT_C128}) {
        if (!(prec_mask & prec)) continue;
        lt_status st = prepare_forward_tables(*p, prec, nullptr);
        if (st == LT_OK) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) st = fail(LT_E_HIP, std::string("table build: ") + hipGetErrorString(e));
        }
        if (st != LT_OK) {
            lattice_plan_destroy(p);
            return st;
        }
    }
    *out = p;
    return LT_OK;
}

lt_status lattice_plan_info(const lt_plan *p, lt_plan_info *info)
{
    if (!p || !info) return fail(LT_E_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->d = p->d;
    info->r = p->r;
    for (int i = 0; i < 4; ++i) info->n[i] = i < p->r ? p->n[i] : 0;
    info->N = p->N;
    info->n_index = p->n_index;
    info->n_completed = p->n_completed;
    info->max_s = p->max_s;
    const Sched &s = p->sched[0][LT_C64].ok ? p->sched[0][LT_C64] : p->sched[0][LT_C128];
    info->bluestein = s.bluestein ? 1 : 0;
    info->passes = s.passes;
    info->fft_len = s.L;
    info->L1 = s.L1;
    info->L2 = s.L2;
    info->cols = s.cols;
    info->rows = s.rows;
    info->L3 = s.L3;
    info->swapped = (p->sched[0][LT_C64].ok ? p->sched[2][LT_C64] : p->sched[2][LT_C128]).ok ? 1 : 0;
    return LT_OK;
}

lt_status lattice_plan_keys(const lt_plan *p, int64_t *key_of_h, int64_t *s_of_key, int32_t *h_of_key)
{
    if (!p) return fail(LT_E_ARG, "plan is NULL");
    if (key_of_h && !p->key_of_h.empty())
        std::memcpy(key_of_h, p->key_of_h.data(), p->key_of_h.size() * sizeof(int64_t));
    if (s_of_key) std::memcpy(s_of_key, p->s_of_key.data(), p->s_of_key.size() * sizeof(int64_t));
    if (h_of_key) std::memcpy(h_of_key, p->h_of_key.data(), p->h_of_key.size() * sizeof(int32_t));
    return LT_OK;
}

lt_status lattice_plan_points(const lt_plan *p, int64_t first, int64_t count, int64_t *num)
{
    if (!p || (!num && count > 0)) return fail(LT_E_ARG, "NULL argument");
    if (first < 0 || count < 0 || first + count > p->N) return fail(LT_E_ARG, "point range out of bounds");
    std::vector<int64_t> k(p->r);
    for (int64_t kappa = first; kappa < first + count; ++kappa) {
        int64_t rem = kappa;
        for (int i = p->r - 1; i >= 0; --i) { k[i] = rem % p->n[i]; rem /= p->n[i]; }
        for (int j = 0; j < p->d; ++j) {
            __int128 acc = 0;
            for (int i = 0; i < p->r; ++i) {
                __int128 zi = p->Z[(size_t)i * p->d + j] % p->n[i];
                if (zi < 0) zi += p->n[i];
                acc += (zi * k[i] % p->n[i]) * (p->N / p->n[i]);
            }
            num[(kappa - first) * p->d + j] = (int64_t)(acc % p->N);
        }
    }
    return LT_OK;
}

void lattice_plan_destroy(lt_plan *p)
{
    if (!p) return;
    for (auto &row : p->dev)
        for (auto &D : row) {
            hipFree(D.twa);
            hipFree(D.twb);
            hipFree(D.tw4hi);
            hipFree(D.tw4lo);
            hipFree(D.s_key);
            hipFree(D.s_row);
            hipFree(D.bhat);
            hipFree(D.twc);
            hipFree(D.tw4hi2);
            hipFree(D.tw4lo2);
        }
    delete p;
}

lt_status strang_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, int32_t shared_v,
                                size_t *bytes)
{
    if (!p || !bytes) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (batch < 0) return fail(LT_E_ARG, "batch must be >= 0");
    *bytes = run_layout(*p, p->sched[0][prec], prec, batch, shared_v != 0).total;
    if (p->sched[2][prec].ok)
        *bytes = std::max(*bytes, swap_layout(*p, p->sched[2][prec], prec, batch, shared_v != 0).total);
    return LT_OK;
}

lt_status strang_adjoint_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, int32_t shared_v,
                                        size_t *bytes)
{
    if (!p || !bytes) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (batch < 0) return fail(LT_E_ARG, "batch must be >= 0");
    *bytes = adj_layout(*p, p->sched[adj_slot(*p, prec)][prec], prec, batch, shared_v != 0).total;
    return LT_OK;
}

}  // extern "C"

namespace {
lt_status run_forward(const lt_plan *cp, lt_prec prec, int32_t batch, const double *v, int64_t v_stride, void *u,
                      double gamma, double dt, int64_t steps, void *ckpt, int64_t ckpt_every, double *sums,
                      void *work, size_t work_bytes, void *stream)
{
    lt_status st = check_common(cp, prec, batch, gamma, dt, steps);
    if (st) return st;
    lt_plan &p = *const_cast<lt_plan *>(cp);
    if (batch == 0) return LT_OK;
    if (!v || !u) {
        if (steps == 0 && !sums) return LT_OK;
        return fail(LT_E_ARG, "v and u must not be NULL");
    }
    if (v_stride != 0 && v_stride < p.N) return fail(LT_E_ARG, "v_stride must be 0 or >= N");
    if (ckpt && ckpt_every < 1) return fail(LT_E_ARG, "ckpt_every must be >= 1 with a checkpoint buffer");
    hipStream_t hs = (hipStream_t)stream;
    if (steps == 0) {
        if (!sums) return LT_OK;
        // no step: the sums of u(0) alone
        if ((st = ensure_device_tables(p, 0, prec, stream))) return st;
        Scratch sc;
        const int nb = diag_partials();
        if ((st = get_work(sc, work, work_bytes, align_up((size_t)batch * nb * 16), hs))) return st;
        double *pp = (double *)sc.ptr;
        HIP_TRY(launch_sums(prec, u, p.N, p.N, batch, nullptr, v, v_stride, pp, hs), "step sums");
        HIP_TRY(launch_step_sums_finish(pp, nb, batch, 0, 1, 0, 1.0 / (double)p.N, 1.0 / (gamma * (double)p.N), sums,
                                        hs),
                "step sums");
        return LT_OK;
    }
    if (p.sched[2][prec].ok)
        return swapped_forward(p, prec, batch, v, v_stride, u, gamma, dt, steps, ckpt, ckpt_every, sums, work,
                               work_bytes, stream);
    if ((st = ensure_device_tables(p, 0, prec, stream))) return st;
    const Sched &s = p.sched[0][prec];
    const DevTables &D = p.dev[0][prec];
    const RunWork L = run_layout(p, s, prec, batch, v_stride == 0);
    const size_t need = L.total + (sums ? sum_bytes(s, batch, steps) : 0);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, need, hs))) return st;
    const SumSink sink = make_sink(s, batch, steps, p.N, gamma, at(sc.ptr, L.total), sums);
    double *ktab = (double *)at(sc.ptr, L.ktab);
    if ((st = make_ktab(p, s, ktab, gamma, dt, hs))) return st;
    if (s.passes == 1) {
        ResArgs a;
        std::memset(&a, 0, sizeof(a));
        a.u = u;
        a.u_bs = p.N;
        a.N = p.N;
        a.L = s.L;
        a.rank2 = s.rank2 ? 1 : 0;
        a.n1 = s.L1;
        a.n2 = s.L2;
        a.ra = s.ra;
        a.rb = s.rb;
        a.twa = D.twa;
        a.twb = D.twb;
        a.bluestein = s.bluestein ? 1 : 0;
        a.s = D.s_key;
        a.ktab = ktab;
        a.bhat = D.bhat;
        a.v = v;
        a.v_bs = v_stride;
        a.phase_half = dt / (2.0 * gamma);
        a.steps = steps;
        a.ck = ckpt;
        a.ck_every = ckpt ? ckpt_every : 0;
        a.ck_stride = (int64_t)batch * p.N;
        a.batch = batch;
        a.sum_part = sink.part;
        HIP_TRY(launch_resident(prec, s, a, batch, hs), "resident run");
        return sums_after(sink, steps, hs);
    }
    if (ckpt)
        HIP_TRY(hipMemcpyAsync(ckpt, u, (size_t)batch * p.N * esz(prec), hipMemcpyDeviceToDevice, hs),
                "checkpoint 0");
    if (s.passes == 3)
        return three_level_forward(p, s, D, prec, batch, v, v_stride, u, gamma, dt, steps, ckpt, ckpt_every,
                                   ktab, at(sc.ptr, L.ptab), hs, sink);
    void *conv = nullptr;
    if (steps >= kConvMinSteps && conv_available(p, 0, s)) {
        if ((st = ensure_device_tables(p, 0, LT_C128, stream))) return st;
        conv = at(sc.ptr, L.conv);
        if ((st = conv_spectrum(p, 0, ktab, conv, at(sc.ptr, L.conv_tmp), hs))) return st;
    }
    return two_pass_forward(p, s, D, prec, batch, v, v_stride, u, gamma, dt, steps, ckpt, ckpt_every,
                            ktab, at(sc.ptr, L.w), at(sc.ptr, L.ptab), conv, hs, false, sink,
                            conv && prec == LT_C64 ? at(sc.ptr, L.conv_f) : nullptr);
}
}  // namespace

extern "C" {

lt_status strang_run(const lt_plan *p, lt_prec prec, int32_t batch, const double *v, int64_t v_stride, void *u,
                     double gamma, double dt, int64_t steps, void *ckpt, int64_t ckpt_every, void *work,
                     size_t work_bytes, void *stream)
{
    return run_forward(p, prec, batch, v, v_stride, u, gamma, dt, steps, ckpt, ckpt_every, nullptr, work,
                       work_bytes, stream);
}

lt_status strang_run_sums_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, int32_t shared_v,
                                         int64_t steps, size_t *bytes)
{
    if (!p || !bytes) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (batch < 0 || steps < 0) return fail(LT_E_ARG, "batch and steps must be >= 0");
    const int w = p->sched[2][prec].ok ? 2 : 0;
    size_t run = 0;
    lt_status st = strang_workspace_size(p, prec, batch, shared_v, &run);
    if (st) return st;
    if (steps == 0) {
        *bytes = align_up((size_t)batch * diag_partials() * 16);
        return LT_OK;
    }
    const size_t base = w == 2 ? swap_layout(*p, p->sched[2][prec], prec, batch, shared_v != 0).total
                               : run_layout(*p, p->sched[0][prec], prec, batch, shared_v != 0).total;
    *bytes = base + sum_bytes(p->sched[w][prec], batch, steps);
    (void)run;
    return LT_OK;
}

lt_status strang_run_sums(const lt_plan *p, lt_prec prec, int32_t batch, const double *v, int64_t v_stride,
                          void *u, double gamma, double dt, int64_t steps, void *ckpt, int64_t ckpt_every,
                          double *sums, void *work, size_t work_bytes, void *stream)
{
    if (!sums) return fail(LT_E_ARG, "sums must not be NULL");
    return run_forward(p, prec, batch, v, v_stride, u, gamma, dt, steps, ckpt, ckpt_every, sums, work, work_bytes,
                       stream);
}

lt_status strang_adjoint(const lt_plan *cp, lt_prec prec, int32_t batch, const double *v, int64_t v_stride,
                         const void *uT, const void *gT, double gamma, double dt, int64_t steps,
                         const void *ckpt, int64_t ckpt_every, void *g0, double *gv, void *work,
                         size_t work_bytes, void *stream)
{
    lt_status st = check_common(cp, prec, batch, gamma, dt, steps);
    if (st) return st;
    lt_plan &p = *const_cast<lt_plan *>(cp);
    if (batch == 0) return LT_OK;
    if (!v || !uT || !gT || !g0 || !gv) return fail(LT_E_ARG, "NULL argument");
    if (v_stride != 0 && v_stride < p.N) return fail(LT_E_ARG, "v_stride must be 0 or >= N");
    const bool shared = v_stride == 0;
    hipStream_t hs = (hipStream_t)stream;
    const size_t S = esz(prec);
    const int64_t N = p.N;
    if (steps == 0) {
        HIP_TRY(hipMemcpyAsync(g0, gT, (size_t)batch * N * S, hipMemcpyDeviceToDevice, hs), "copy");
        HIP_TRY(hipMemsetAsync(gv, 0, (size_t)(shared ? 1 : batch) * N * sizeof(double), hs), "memset");
        return LT_OK;
    }
    if (!ckpt || ckpt_every < 1) return fail(LT_E_ARG, "the adjoint needs the forward checkpoints");
    const int slot = adj_slot(p, prec);
    if ((st = ensure_device_tables(p, slot, prec, stream))) return st;
    const Sched &s = p.sched[slot][prec];
    const DevTables &D = p.dev[slot][prec];
    const AdjWork L = adj_layout(p, s, prec, batch, shared);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, L.total, hs))) return st;
    // a swapped rank-2 schedule sweeps the transposed tensor (n2 x n1): u(T),
    // the cotangent and v are transposed into the workspace, the checkpoint
    // resets read the lattice-order checkpoints transposed, and dJ/du0 and
    // dJ/dv are transposed back at the end
    const int n1 = s.L2, n2 = s.L1;
    if (s.swapped) {
        void *UT = at(sc.ptr, L.ut), *GT = at(sc.ptr, L.gt);
        double *VT = (double *)at(sc.ptr, L.vt);
        HIP_TRY(launch_transpose((int)S, UT, uT, batch, n1, n2, N, N, hs), "state transpose");
        HIP_TRY(launch_transpose((int)S, GT, gT, batch, n1, n2, N, N, hs), "cotangent transpose");
        HIP_TRY(launch_transpose(8, VT, v, shared ? 1 : batch, n1, n2, N, shared ? N : v_stride, hs),
                "potential transpose");
        uT = UT;
        gT = GT;
        v = VT;
        v_stride = shared ? 0 : N;
    }
    void *W = at(sc.ptr, L.w);
    double *gacc = (double *)at(sc.ptr, L.gacc);
    double *ktab = (double *)at(sc.ptr, L.ktab);
    const double dtb = -dt;  // the backward sweep runs the scheme with -dt
    const double halfb = dtb / (2.0 * gamma);
    if ((st = make_ktab(p, s, ktab, gamma, dtb, hs))) return st;
    // the backward sweep's kinetic part F^-1 conj(K) F as one cyclic convolution
    const void *conv = nullptr;
    if (steps >= kConvMinSteps && conv_available(p, slot, s)) {
        if ((st = ensure_device_tables(p, slot, LT_C128, stream))) return st;
        if ((st = conv_spectrum(p, slot, ktab, at(sc.ptr, L.conv), at(sc.ptr, L.conv_tmp), hs))) return st;
        conv = at(sc.ptr, L.conv);
    }
    const bool chirpz = s.bluestein && !conv;
    HIP_TRY(hipMemsetAsync(gacc, 0, (size_t)batch * N * sizeof(double), hs), "memset");
    const double c = dt / (2.0 * gamma);
    // the backward merged potential step exp(-i 2 halfb v) of the interior
    // merge passes, as a per-point table
    void *ptab = at(sc.ptr, L.ptab);
    if (steps > 1)
        HIP_TRY(launch_phase_table(prec, ptab, v, v_stride, shared ? 1 : batch, N, 2.0 * halfb, hs),
                "potential table");
    void *Wg = at(W, (size_t)batch * s.L * S);

    ColArgs base = col_base(s, D, N);
    base.C = std::max(1, s.cols / 2);
    base.ntiles = (s.L2 + base.C - 1) / base.C;
    base.buf = W;
    base.buf_bs = s.L;
    base.buf2 = Wg;
    base.buf2_bs = s.L;
    base.v = v;
    base.v_bs = v_stride;
    base.chirp = chirpz ? 1 : 0;
    base.gacc = gacc;
    base.gacc_bs = N;
    base.reset_phase = c;
    base.reset_bs = N;

    ColArgs first = base;
    first.adjoint = 1;
    first.phase = halfb;
    first.in = uT;
    first.in_bs = N;
    first.in2 = gT;
    first.in2_bs = N;
    first.post_fwd = 1;
    first.gcoef = c;
    HIP_TRY(launch_col(prec, s, first, batch, hs), "adjoint column pass");

    RowArgs r = row_base(s, D);
    r.buf = W;
    r.buf_bs = s.L;
    if (conv) {
        r.bhat = (const double *)conv;
        if (prec == LT_C64) {  // as in the forward run: the complex64 rows read it in complex float
            HIP_TRY(launch_spectrum_f32(at(sc.ptr, L.conv_f), conv, s.L, hs), "convolution spectrum (complex float)");
            r.bhat_f = (const float *)at(sc.ptr, L.conv_f);
        }
    } else if (s.bluestein) {
        r.bhat = D.bhat;
    } else {
        r.s = D.s_row;
        r.ktab = ktab;
    }
    ColArgs kinp = col_base(s, D, N);
    kinp.buf = W;
    kinp.buf_bs = s.L;
    kinp.pre_inv = 1;
    kinp.post_fwd = 1;
    kinp.s = D.s_key;
    kinp.ktab = ktab;
    for (int64_t j = steps; j >= 1; --j) {
        r.conj_tab = 0;
        HIP_TRY(launch_row(prec, s, r, 2 * batch, hs), "adjoint row pass");
        if (chirpz) {
            HIP_TRY(launch_col(prec, s, kinp, 2 * batch, hs), "adjoint column pass (kinetic)");
            r.conj_tab = 1;
            HIP_TRY(launch_row(prec, s, r, 2 * batch, hs), "adjoint row pass");
        }
        const int64_t k = j - 1;  // state index at this merge point
        ColArgs m = base;
        m.pre_inv = 1;
        if (k % ckpt_every == 0) {
            m.reset = (const char *)ckpt + (size_t)(k / ckpt_every) * batch * N * S;
            m.reset_t = s.swapped ? 1 : 0;
        }
        if (k > 0) {
            m.adjoint = 2;
            m.phase = 2.0 * halfb;
            m.post_fwd = 1;
            m.gcoef = 2.0 * c;
            if (!m.reset) {
                m.ptab = ptab;
                m.ptab_bs = shared ? 0 : N;
            }
        } else {
            m.adjoint = 3;
            m.phase = halfb;
            m.out2 = s.swapped ? at(sc.ptr, L.ut) : g0;  // u(T) was read by the first pass
            m.out2_bs = N;
            m.gcoef = c;
        }
        HIP_TRY(launch_col(prec, s, m, batch, hs), "adjoint column pass");
    }
    if (s.swapped) {
        HIP_TRY(launch_transpose((int)S, g0, at(sc.ptr, L.ut), batch, n2, n1, N, N, hs), "gradient transpose");
        if (shared) {
            double *GV = (double *)at(sc.ptr, L.gt);  // the cotangent was read by the first pass
            HIP_TRY(launch_reduce_batch(GV, gacc, N, batch, hs), "gradient reduction");
            HIP_TRY(launch_transpose(8, gv, GV, 1, n2, n1, N, N, hs), "gradient transpose");
        } else {
            HIP_TRY(launch_transpose(8, gv, gacc, batch, n2, n1, N, N, hs), "gradient transpose");
        }
        return LT_OK;
    }
    if (shared) {
        HIP_TRY(launch_reduce_batch(gv, gacc, N, batch, hs), "gradient reduction");
    } else {
        HIP_TRY(hipMemcpyAsync(gv, gacc, (size_t)batch * N * sizeof(double), hipMemcpyDeviceToDevice, hs),
                "copy");
    }
    return LT_OK;
}

lt_status strang_batched_workspace_size(int32_t B, const lt_plan *const *plans, lt_prec prec, size_t *bytes)
{
    if (B < 0 || (B > 0 && !plans) || !bytes) return fail(LT_E_ARG, "bad arguments");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    for (int i = 0; i < B; ++i)
        if (!plans[i]) return fail(LT_E_ARG, "plan is NULL");
    *bytes = B ? batch_layout(B, plans, prec).total : 0;
    return LT_OK;
}

}  // extern "C"

namespace {
// Everything the launches of a batch need, built once: host copies of the
// descriptors (kinetic tables, resident problems, two-pass problems, class
// lists) and the device-side tables, all pointing into one workspace.
struct BatchRun {
    int prec = 0;
    BatchLayout BL;
    std::vector<KtabDesc> kd;
    std::vector<ResArgs> res;
    std::vector<BatchDesc> two;
    std::vector<MemberList> cols, rows;  // [0] general kernel, then one per register-staged length
    std::vector<int> lists;
    struct ConvJob {
        lt_plan *p;
        const double *ktab;
        void *G, *tmp;
        void *Gf;  // complex64 batches: the spectrum rounded to complex float, or null
        int64_t L;
    };
    std::vector<ConvJob> conv_jobs;
    size_t lds_res = 0, lds_col = 0, lds_row = 0;
    int64_t max_ktab = 0, gmax = 0;
};

lt_status batch_check(int32_t B, const lt_plan *const *plans, lt_prec prec, const double *const *v, void *const *u,
                      const double *gamma, const double *dt, const int64_t *steps)
{
    if (B < 0) return fail(LT_E_ARG, "B must be >= 0");
    if (B == 0) return LT_OK;
    if (!plans || !v || !u || !gamma || !dt || !steps) return fail(LT_E_ARG, "NULL argument");
    lt_status st;
    for (int i = 0; i < B; ++i) {
        if ((st = check_common(plans[i], prec, 1, gamma[i], dt[i], steps[i]))) return st;
        if (steps[i] > 0 && (!v[i] || !u[i])) return fail(LT_E_ARG, "v and u must not be NULL");
    }
    return LT_OK;
}

// Host descriptors of a batch whose workspace starts at ws; enqueues the
// members' potential tables (they read only v).
lt_status batch_build(int32_t B, const lt_plan *const *plans, lt_prec prec, const double *const *v, void *const *u,
                      const double *gamma, const double *dt, const int64_t *steps, void *ws, BatchRun &R,
                      hipStream_t hs)
{
    lt_status st;
    R.prec = prec;
    R.BL = batch_layout(B, plans, prec);
    const size_t S = esz(prec);
    for (int i = 0; i < B; ++i) {
        if (steps[i] == 0) continue;
        lt_plan &p = *const_cast<lt_plan *>(plans[i]);
        if ((st = ensure_device_tables(p, 0, prec, hs))) return st;
        const Sched &s = p.sched[0][prec];
        const DevTables &D = p.dev[0][prec];
        const RunWork L = run_layout(p, s, prec, 1, true, true, true);
        char *w = at(ws, R.BL.off[i]);
        double *ktab = (double *)(w + L.ktab);
        R.kd.push_back({ktab, p.max_s + 1, kinetic_angle(gamma[i], dt[i]), s.bluestein ? 1.0 : 1.0 / (double)s.L});
        R.max_ktab = std::max<int64_t>(R.max_ktab, p.max_s + 1);
        const double half = dt[i] / (2.0 * gamma[i]);
        if (s.passes == 1) {
            ResArgs a;
            std::memset(&a, 0, sizeof(a));
            a.u = u[i];
            a.u_bs = p.N;
            a.N = p.N;
            a.L = s.L;
            a.rank2 = s.rank2 ? 1 : 0;
            a.n1 = s.L1;
            a.n2 = s.L2;
            a.ra = s.ra;
            a.rb = s.rb;
            a.twa = D.twa;
            a.twb = D.twb;
            a.bluestein = s.bluestein ? 1 : 0;
            a.s = D.s_key;
            a.ktab = ktab;
            a.bhat = D.bhat;
            a.v = v[i];
            a.phase_half = half;
            a.steps = steps[i];
            a.batch = 1;
            R.res.push_back(a);
            R.lds_res = std::max(R.lds_res, (size_t)s.L * S);
            continue;
        }
        if (s.L2 > kTileElems || s.passes == 3)
            return fail(LT_E_UNSUPPORTED, "batch members take transforms of at most 4096 x 4096 points");
        // the merged potential step exp(-i dt v / gamma) of the interior column
        // passes, as a per-point table
        void *ptab = steps[i] > 1 ? (void *)(w + L.ptab) : nullptr;
        if (ptab)
            HIP_TRY(launch_phase_table(prec, ptab, v[i], 0, 1, p.N, 2.0 * half, hs), "potential table");
        Roles Ro = two_pass_roles(s, D, p.N, v[i], 0, u[i], w + L.w, half, ktab, ptab);
        // chirp-z problems of 4 steps or more: the convolution form (spectrum
        // built once the kinetic tables exist)
        const bool conv = steps[i] >= kConvMinSteps && conv_available(p, 0, s);
        if (conv) {
            if ((st = ensure_device_tables(p, 0, LT_C128, hs))) return st;
            void *Gf = prec == LT_C64 ? (void *)(w + L.conv_f) : nullptr;
            R.conv_jobs.push_back({&p, ktab, w + L.conv, w + L.conv_tmp, Gf, s.L});
            if (Gf) Ro.row.bhat_f = (const float *)Gf;
            Ro.first.chirp = 0;
            Ro.last.chirp = 0;
            Ro.row.bhat = (const double *)(w + L.conv);
        }
        BatchDesc b;
        std::memset(&b, 0, sizeof(b));
        b.col[0] = Ro.first;
        b.col[1] = Ro.pot;
        b.col[2] = Ro.kin;
        b.col[3] = Ro.last;
        b.row[0] = Ro.row;
        b.row[1] = Ro.row;
        b.row[1].conj_tab = 1;
        b.bluestein = (s.bluestein && !conv) ? 1 : 0;
        b.npass = (b.bluestein ? 4 : 2) * steps[i] + 1;
        R.two.push_back(b);
        R.lds_col = std::max(R.lds_col, (size_t)Ro.first.L1 * Ro.first.C * S);
        R.lds_row = std::max(R.lds_row, (size_t)Ro.row.rows * Ro.row.L2 * S);
    }
    // longest schedules first: the problems still running at pass g are a prefix
    std::stable_sort(R.two.begin(), R.two.end(),
                     [](const BatchDesc &a, const BatchDesc &b) { return a.npass > b.npass; });
    const int n2 = (int)R.two.size();
    R.gmax = n2 ? R.two[0].npass : 0;
    // column and row kernel classes: register-staged passes where the length
    // has one (two passes per step only), the general kernel otherwise
    R.cols.assign(1, MemberList());
    R.rows.assign(1, MemberList());
    R.cols[0].key = R.rows[0].key = -1;
    auto list_for = [](std::vector<MemberList> &ls, int key) -> MemberList & {
        for (auto &l : ls)
            if (l.key == key) return l;
        ls.emplace_back();
        ls.back().key = key;
        return ls.back();
    };
    for (int i = 0; i < n2; ++i) {
        const BatchDesc &b = R.two[i];
        const ColArgs &pc = b.col[1];
        const RowArgs &pr = b.row[0];
        const bool fc = !b.bluestein && pc.v && fast_col_fits(prec, 1, pc.L1, pc.L2, pc.C);
        const bool fr = !b.bluestein && fast_row_fits(prec, 1, pr.L1, pr.L2, pr.rows);
        MemberList &lc = fc ? list_for(R.cols, pc.L1) : R.cols[0];
        MemberList &lr = fr ? list_for(R.rows, 2 * pr.L2 + (pr.bhat ? 0 : 1)) : R.rows[0];
        lc.mem.push_back(i);
        lc.npass.push_back(b.npass);
        lr.mem.push_back(i);
        lr.npass.push_back(b.npass);
    }
    if ((int)(R.cols.size() + R.rows.size()) > kMaxBatchLists) return fail(LT_E_UNSUPPORTED, "too many kernel classes");
    for (auto *ls : {&R.cols, &R.rows}) {
        const bool is_col = ls == &R.cols;
        for (auto &l : *ls) {
            l.start.assign(1, 0);
            for (int i : l.mem)
                l.start.push_back(l.start.back() + (is_col ? R.two[i].col[0].ntiles : R.two[i].row[0].nblk));
            l.idx_off = R.lists.size();
            R.lists.insert(R.lists.end(), l.mem.begin(), l.mem.end());
            l.start_off = R.lists.size();
            R.lists.insert(R.lists.end(), l.start.begin(), l.start.end());
            l.act = (int)l.mem.size();
        }
    }
    return LT_OK;
}

// multiplier of a register-staged row class (key = 2 L2 + kind): 1 the kinetic
// table; 0 the convolution spectrum, which complex64 batches read in complex
// float (every member of such a class has the convolution form and its
// rounded copy, batch_build)
int row_mid(int prec, int key)
{
    const int kind = key % 2;
    return kind == 0 && prec == LT_C64 ? 2 : kind;
}

// the descriptor block as uploaded
std::vector<char> batch_blob(const BatchRun &R)
{
    std::vector<char> blob(R.BL.desc_bytes, 0);
    std::memcpy(blob.data() + R.BL.d_ktab, R.kd.data(), R.kd.size() * sizeof(KtabDesc));
    if (!R.res.empty()) std::memcpy(blob.data() + R.BL.d_res, R.res.data(), R.res.size() * sizeof(ResArgs));
    if (!R.two.empty()) std::memcpy(blob.data() + R.BL.d_two, R.two.data(), R.two.size() * sizeof(BatchDesc));
    std::memcpy(blob.data() + R.BL.d_lists, R.lists.data(), R.lists.size() * sizeof(int));
    return blob;
}

// kinetic tables and convolution spectra (after the descriptor upload)
lt_status batch_tables(const BatchRun &R, char *dd, hipStream_t hs)
{
    lt_status st;
    HIP_TRY(launch_ktab_multi((const KtabDesc *)(dd + R.BL.d_ktab), (int)R.kd.size(), R.max_ktab, hs),
            "kinetic tables");
    for (const auto &j : R.conv_jobs) {
        if ((st = conv_spectrum(*j.p, 0, j.ktab, j.G, j.tmp, hs))) return st;
        if (j.Gf) HIP_TRY(launch_spectrum_f32(j.Gf, j.G, j.L, hs), "convolution spectrum (complex float)");
    }
    return LT_OK;
}

// The pass launches of one batch run.  Problems that fit one workgroup run
// their whole step loop in one launch on rs (a second stream joined through
// the two events, or hs itself), overlapped with the pass-by-pass launches of
// the others on hs.  Enqueues kernels and event operations only.
lt_status batch_passes(const BatchRun &R, char *dd, hipStream_t hs, hipStream_t rs, hipEvent_t ev_fork,
                       hipEvent_t ev_join)
{
    const int prec = R.prec;
    const int n2 = (int)R.two.size();
    const bool fork = !R.res.empty() && n2 && rs != hs;
    if (fork) {
        HIP_TRY(hipEventRecord(ev_fork, hs), "event record");
        HIP_TRY(hipStreamWaitEvent(rs, ev_fork, 0), "stream wait");
    }
    if (!R.res.empty())
        HIP_TRY(launch_resident_multi(prec, (const ResArgs *)(dd + R.BL.d_res), (int)R.res.size(), R.lds_res,
                                      fork ? rs : hs),
                "resident batch");
    const BatchDesc *dtwo = (const BatchDesc *)(dd + R.BL.d_two);
    const int *dl = (const int *)(dd + R.BL.d_lists);
    std::vector<MemberList> cols = R.cols, rows = R.rows;  // act counts down per run
    int herr = 0;
    for (int64_t g = 0; g < R.gmax && !herr; ++g) {
        const bool col = !(g & 1);
        for (auto &l : col ? cols : rows) {
            while (l.act > 0 && l.npass[l.act - 1] <= g) --l.act;
            if (herr || l.act == 0) continue;
            const int *idx = dl + l.idx_off, *start = dl + l.start_off;
            if (!col) {
                herr = l.key < 0 ? launch_row_multi(prec, dtwo, idx, start, l.act, l.start[l.act], 0, g, R.lds_row, hs)
                                 : launch_row_fast_multi(prec, l.var, l.key / 2, row_mid(prec, l.key), dtwo, idx, start, l.act,
                                                         l.start[l.act], 0, g, hs);
                continue;
            }
            if (l.key < 0) {  // general kernel: every role
                herr = launch_col_multi(prec, dtwo, idx, start, l.act, l.start[l.act], 0, g, R.lds_col, hs);
                continue;
            }
            if (g == 0) {  // every member's first pass
                herr = launch_col_fast_multi(prec, l.var, l.key, 9, dtwo, idx, start, l.act, l.start[l.act], 0, g, hs);
                continue;
            }
            // register-staged interior passes, then the last pass of the
            // members whose schedules end here (a contiguous range [a, act))
            herr = launch_col_fast_multi(prec, l.var, l.key, 0, dtwo, idx, start, l.act, l.start[l.act], 0, g, hs);
            int a = l.act;
            while (a > 0 && l.npass[a - 1] == g + 1) --a;
            if (!herr && a < l.act)
                herr = launch_col_fast_multi(prec, l.var, l.key, 10, dtwo, idx, start, l.act,
                                             l.start[l.act] - l.start[a], l.start[a], g, hs);
        }
    }
    if (fork) {  // join even after a failed launch: the workspace must outlive the second stream's work
        int e = (int)hipEventRecord(ev_join, rs);
        if (!e) e = (int)hipStreamWaitEvent(hs, ev_join, 0);
        if (e) hipStreamSynchronize(rs);
        if (!herr) herr = e;
    }
    HIP_TRY(herr, "batched pass");
    return LT_OK;
}
}  // namespace

extern "C" {

lt_status strang_run_batched(int32_t B, const lt_plan *const *plans, lt_prec prec, const double *const *v,
                             void *const *u, const double *gamma, const double *dt, const int64_t *steps,
                             void *work, size_t work_bytes, void *stream)
{
    lt_status st = batch_check(B, plans, prec, v, u, gamma, dt, steps);
    if (st || B == 0) return st;
    hipStream_t hs = (hipStream_t)stream;
    const BatchLayout BL = batch_layout(B, plans, prec);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, BL.total, hs))) return st;
    BatchRun R;
    if ((st = batch_build(B, plans, prec, v, u, gamma, dt, steps, sc.ptr, R, hs))) return st;
    if (R.kd.empty()) return LT_OK;
    const std::vector<char> blob = batch_blob(R);
    char *dd = at(sc.ptr, BL.desc);
    if ((st = upload_async(dd, blob.data(), blob.size(), hs))) return st;
    if ((st = batch_tables(R, dd, hs))) return st;
    hipStream_t rs = hs;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    if (!R.res.empty() && !R.two.empty()) {
        if ((st = side_stream(&rs))) return st;
        HIP_TRY(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming), "event");
        HIP_TRY(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming), "event");
    }
    st = batch_passes(R, dd, hs, rs, ev_fork, ev_join);
    if (ev_fork) hipEventDestroy(ev_fork);
    if (ev_join) hipEventDestroy(ev_join);
    return st;
}

// ---------------------------------------------------------------- batch objects
struct lt_batch {
    BatchRun R;
    void *mem = nullptr;    // workspace and descriptor block (device, owned)
    char *dd = nullptr;     // descriptor block
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int device = -1;
};

lt_status strang_batch_create(int32_t B, const lt_plan *const *plans, lt_prec prec, const double *const *v,
                              void *const *u, const double *gamma, const double *dt, const int64_t *steps,
                              void *stream, lt_batch **out)
{
    if (!out) return fail(LT_E_ARG, "out is NULL");
    *out = nullptr;
    lt_status st = batch_check(B, plans, prec, v, u, gamma, dt, steps);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    std::unique_ptr<lt_batch> b(new (std::nothrow) lt_batch());
    if (!b) return fail(LT_E_NOMEM, "batch object");
    HIP_TRY(hipGetDevice(&b->device), "device query");
    if (B > 0) {
        const BatchLayout BL = batch_layout(B, plans, prec);
        HIP_TRY(hipMalloc(&b->mem, BL.total), "batch workspace");
        auto release = [&]() {
            hipFree(b->mem);
            b->mem = nullptr;
        };
        if ((st = batch_build(B, plans, prec, v, u, gamma, dt, steps, b->mem, b->R, hs))) {
            hipStreamSynchronize(hs);
            release();
            return st;
        }
        b->dd = at(b->mem, BL.desc);
        if (!b->R.kd.empty()) {
            const std::vector<char> blob = batch_blob(b->R);
            hipError_t e = hipMemcpyAsync(b->dd, blob.data(), blob.size(), hipMemcpyHostToDevice, hs);
            if (e == hipSuccess) st = batch_tables(b->R, b->dd, hs);
            const hipError_t e2 = hipStreamSynchronize(hs);  // blob is host memory of this frame
            if (e == hipSuccess) e = e2;
            if (!st && e != hipSuccess) st = fail(LT_E_HIP, std::string("batch tables: ") + hipGetErrorString(e));
            if (st) {
                release();
                return st;
            }
        }
        if (!b->R.res.empty() && !b->R.two.empty()) {
            HIP_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking), "stream");
            HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "event");
            HIP_TRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming), "event");
        }
    }
    *out = b.release();
    return LT_OK;
}

lt_status strang_batch_run(const lt_batch *b, void *stream)
{
    if (!b) return fail(LT_E_ARG, "batch is NULL");
    if (b->R.kd.empty()) return LT_OK;
    hipStream_t hs = (hipStream_t)stream;
    return batch_passes(b->R, b->dd, hs, b->side ? b->side : hs, b->ev_fork, b->ev_join);
}

lt_status strang_batch_autotune(lt_batch *b, int32_t reps, void *stream)
{
    if (!b) return fail(LT_E_ARG, "batch is NULL");
    if (reps < 1) return fail(LT_E_ARG, "reps must be >= 1");
    BatchRun &R = b->R;
    if (R.two.empty()) return LT_OK;
    hipStream_t hs = (hipStream_t)stream;
    const size_t S = esz(R.prec);
    // a copy of the two-pass descriptors whose transform buffers point into
    // scratch, so that timing the passes leaves the members' states alone
    std::vector<BatchDesc> tune = R.two;
    size_t bytes = 0;
    std::vector<size_t> off(tune.size());
    for (size_t i = 0; i < tune.size(); ++i) {
        off[i] = bytes;
        bytes += align_up((size_t)tune[i].col[0].L1 * tune[i].col[0].L2 * S);
    }
    const size_t dsz = align_up(tune.size() * sizeof(BatchDesc));
    const size_t lsz = align_up(R.lists.size() * sizeof(int));
    void *scratch = nullptr;
    HIP_TRY(hipMalloc(&scratch, bytes + dsz + lsz), "autotune scratch");
    lt_status st = LT_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int herr = (int)hipMemsetAsync(scratch, 0, bytes, hs);
    for (size_t i = 0; i < tune.size(); ++i) {
        void *buf = at(scratch, off[i]);
        for (auto &c : tune[i].col) {
            c.buf = buf;
            c.buf_bs = 0;
            c.out = nullptr;  // first / last roles never run below
        }
        for (auto &r : tune[i].row) {
            r.buf = buf;
            r.buf_bs = 0;
        }
    }
    BatchDesc *dtwo = (BatchDesc *)at(scratch, bytes);
    int *dl = (int *)at(scratch, bytes + dsz);
    if (!herr) herr = (int)hipMemcpyAsync(dtwo, tune.data(), tune.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, hs);
    if (!herr) herr = (int)hipMemcpyAsync(dl, R.lists.data(), R.lists.size() * sizeof(int), hipMemcpyHostToDevice, hs);
    if (!herr) herr = (int)hipEventCreate(&e0);
    if (!herr) herr = (int)hipEventCreate(&e1);
    if (!herr) herr = (int)hipStreamSynchronize(hs);
    // every member at an interior pass: column g = 2, row g = 1 (members with a
    // single step have no interior column pass and skip it inside the kernel)
    for (int which = 0; which < 2 && !herr; ++which) {
        auto &ls = which == 0 ? R.cols : R.rows;
        for (auto &l : ls) {
            if (l.key < 0 || l.mem.empty() || herr) continue;
            const int *idx = dl + l.idx_off, *start = dl + l.start_off;
            const int nm = (int)l.mem.size(), nb = l.start[nm];
            // 256 x 16 and 512 x 8 on 4096-element tiles; 256 x 8 on
            // 2048-element tiles for lengths up to 2048; three interleaved
            // rounds, the fastest of each variant counts
            const int len = which == 0 ? l.key : l.key / 2;
            const int vars[3] = {1, 2, 5};
            float t[3] = {1e30f, 1e30f, 1e30f};
            for (int round = 0; round < 3 && !herr; ++round) {
                for (int i = 0; i < 3 && !herr; ++i) {
                    const int var = vars[i];
                    if (var == 5 && len > 2048) continue;
                    auto go = [&]() {
                        return which == 0
                                   ? launch_col_fast_multi(R.prec, var, l.key, 0, dtwo, idx, start, nm, nb, 0, 2, hs)
                                   : launch_row_fast_multi(R.prec, var, l.key / 2, row_mid(R.prec, l.key), dtwo, idx,
                                                           start, nm, nb, 0, 1, hs);
                    };
                    herr = go();  // warm-up
                    if (!herr) herr = (int)hipEventRecord(e0, hs);
                    for (int k = 0; k < reps && !herr; ++k) herr = go();
                    if (!herr) herr = (int)hipEventRecord(e1, hs);
                    if (!herr) herr = (int)hipEventSynchronize(e1);
                    float ms = 0.0f;
                    if (!herr) herr = (int)hipEventElapsedTime(&ms, e0, e1);
                    if (!herr) t[i] = std::min(t[i], ms);
                }
            }
            int best = 0;
            for (int i = 1; i < 3; ++i)
                if (t[i] < t[best]) best = i;
            l.var = vars[best];
        }
    }
    if (herr) st = fail(LT_E_HIP, std::string("batch autotune: ") + hipGetErrorString((hipError_t)herr));
    hipStreamSynchronize(hs);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(scratch);
    return st;
}

lt_status strang_batch_kernels(const lt_batch *b, int32_t *ncls, int32_t *key, int32_t *variant, int32_t cap)
{
    if (!b || !ncls) return fail(LT_E_ARG, "NULL argument");
    int n = 0;
    for (int which = 0; which < 2; ++which)
        for (const auto &l : which == 0 ? b->R.cols : b->R.rows) {
            if (l.key < 0 || l.mem.empty()) continue;
            if (n < cap && key && variant) {
                key[n] = which == 0 ? l.key : -l.key;
                variant[n] = l.var;
            }
            ++n;
        }
    *ncls = n;
    return LT_OK;
}

void strang_batch_destroy(lt_batch *b)
{
    if (!b) return;
    int cur = -1;
    hipGetDevice(&cur);
    if (b->device >= 0) hipSetDevice(b->device);
    if (b->mem) hipFree(b->mem);  // waits for the work of the device
    if (b->ev_fork) hipEventDestroy(b->ev_fork);
    if (b->ev_join) hipEventDestroy(b->ev_join);
    if (b->side) hipStreamDestroy(b->side);
    if (cur >= 0) hipSetDevice(cur);
    delete b;
}

// ---------------------------------------------------------------- compositions
// One step of a symmetric composition: Strang steps of dt * w[i], i < P.
// Workspace of a composed run (two-pass slot): per distinct substep a
// kinetic table and (chirp-z) a convolution spectrum, per boundary a merged
// potential table (complex64), the transform buffer (chirp-z) and scratch.
struct ComposedWork {
    size_t ktab[3] = {}, conv[3] = {}, conv_f[3] = {}, ptab[3] = {}, w = 0, tmp = 0, total = 0;
};

ComposedWork composed_layout(const lt_plan &p, const Sched &s, int prec, int batch, bool shared_v, int P)
{
    ComposedWork c;
    size_t off = 0;
    for (int i = 0; i < P; ++i) {
        c.ktab[i] = off;
        off = align_up(off + (size_t)(p.max_s + 1) * 16);
        if (s.bluestein) {
            c.conv[i] = off;
            off = align_up(off + (size_t)s.L * 16);
            if (prec == LT_C64) {  // the spectrum rounded to complex float for the complex64 rows
                c.conv_f[i] = off;
                off = align_up(off + (size_t)s.L * 8);
            }
        }
        c.ptab[i] = off;
        off = align_up(off + (size_t)(shared_v ? 1 : batch) * p.N * 16);
    }
    c.w = off;
    if (s.bluestein) off = align_up(off + (size_t)batch * s.L * esz(prec));
    c.tmp = off;
    if (s.bluestein) off = align_up(off + (size_t)p.N * 16);
    c.total = off;
    return c;
}

// fourth order: the triple jump w1, w0, w1 with w1 = 1 / (2 - 2^(1/3)),
// w0 = 1 - 2 w1 (Yoshida's symmetric composition of a second-order
// symmetric step; local error O(dt^5))
int composition_weights(int order, double *w)
{
    if (order == 2) {
        w[0] = 1.0;
        return 1;
    }
    const double c = std::cbrt(2.0);
    w[0] = w[2] = 1.0 / (2.0 - c);
    w[1] = 1.0 - 2.0 * w[0];
    return 3;
}

// ---------------------------------------------------------------- diagnostics
// workspace: the transform buffer (batch x L), the chirp-z spectrum in natural
// order (batch x N), point and spectral partial sums
struct DiagWork {
    size_t w = 0, nat = 0, pp = 0, ps = 0, total = 0;
};

DiagWork diag_layout(const lt_plan &p, const Sched &s, int prec, int batch)
{
    DiagWork d;
    size_t off = 0;
    d.w = off;
    off = align_up(off + (size_t)batch * s.L * esz(prec));
    d.nat = off;
    if (s.bluestein) off = align_up(off + (size_t)batch * p.N * esz(prec));
    d.pp = off;
    off = align_up(off + (size_t)batch * diag_partials() * 2 * sizeof(double));
    d.ps = off;
    off = align_up(off + (size_t)batch * diag_partials() * 2 * sizeof(double));
    d.total = off;
    return d;
}

lt_status lattice_diagnostics_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, size_t *bytes)
{
    if (!p || !bytes) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (batch < 0) return fail(LT_E_ARG, "batch must be >= 0");
    *bytes = diag_layout(*p, p->sched[1][prec], prec, batch).total;
    return LT_OK;
}

lt_status lattice_diagnostics(const lt_plan *cp, lt_prec prec, int32_t batch, const double *v, int64_t v_stride,
                              const void *u, double gamma, double *out, void *work, size_t work_bytes,
                              void *stream)
{
    lt_status st = check_common(cp, prec, batch, gamma, 0.0, 0);
    if (st) return st;
    lt_plan &p = *const_cast<lt_plan *>(cp);
    if (batch == 0) return LT_OK;
    if (!v || !u || !out) return fail(LT_E_ARG, "v, u and out must not be NULL");
    if (v_stride != 0 && v_stride < p.N) return fail(LT_E_ARG, "v_stride must be 0 or >= N");
    // the two-pass schedule of the adjoint slot exists for every plan
    if ((st = ensure_device_tables(p, 1, prec, stream))) return st;
    const Sched &s = p.sched[1][prec];
    const DevTables &D = p.dev[1][prec];
    hipStream_t hs = (hipStream_t)stream;
    const int64_t N = p.N;
    const DiagWork L = diag_layout(p, s, prec, batch);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, L.total, hs))) return st;
    void *W = at(sc.ptr, L.w);
    double *pp = (double *)at(sc.ptr, L.pp), *ps = (double *)at(sc.ptr, L.ps);
    HIP_TRY(launch_sums(prec, u, N, N, batch, nullptr, v, v_stride, pp, hs), "point sums");
    // U = F u: first column pass (with the chirp for chirp-z), then the rows
    ColArgs c = col_base(s, D, N);
    c.buf = W;
    c.buf_bs = s.L;
    c.in = u;
    c.in_bs = N;
    c.post_fwd = 1;
    c.chirp = s.bluestein ? 1 : 0;
    HIP_TRY(launch_col(prec, s, c, batch, hs), "diagnostics transform");
    RowArgs r = row_base(s, D);
    r.buf = W;
    r.buf_bs = s.L;
    double kscale;
    if (s.bluestein) {
        r.bhat = D.bhat;
        HIP_TRY(launch_row(prec, s, r, batch, hs), "diagnostics transform");
        void *nat = at(sc.ptr, L.nat);
        ColArgs e = col_base(s, D, N);
        e.buf = W;
        e.buf_bs = s.L;
        e.pre_inv = 1;
        e.out = nat;
        e.out_bs = N;
        e.chirp = 1;
        HIP_TRY(launch_col(prec, s, e, batch, hs), "diagnostics transform");  // unitary F u, key order
        HIP_TRY(launch_sums(prec, nat, N, N, batch, D.s_key, nullptr, 0, ps, hs), "spectral sums");
        kscale = 1.0;
    } else {
        r.fft_only = 1;  // unnormalised F u at the row-pass positions
        HIP_TRY(launch_row(prec, s, r, batch, hs), "diagnostics transform");
        HIP_TRY(launch_sums(prec, W, s.L, s.L, batch, D.s_row, nullptr, 0, ps, hs), "spectral sums");
        kscale = 1.0 / (double)N;
    }
    HIP_TRY(launch_diag_finish(pp, ps, batch, N, gamma, kscale, out, hs), "diagnostics");
    return LT_OK;
}

// ---------------------------------------------------------------- projection error
// workspace: the transform buffer, the chirp-z spectrum in key order, partials
lt_status lattice_projection_error_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, size_t *bytes)
{
    return lattice_diagnostics_workspace_size(p, prec, batch, bytes);
}

lt_status lattice_projection_error(const lt_plan *cp, lt_prec prec, int32_t batch, const void *u,
                                   const double *ghat, double *out, void *work, size_t work_bytes, void *stream)
{
    lt_status st = check_common(cp, prec, batch, 1.0, 0.0, 0);
    if (st) return st;
    lt_plan &p = *const_cast<lt_plan *>(cp);
    if (batch == 0) return LT_OK;
    if (!u || !ghat || !out) return fail(LT_E_ARG, "u, ghat and out must not be NULL");
    if ((st = ensure_device_tables(p, 1, prec, stream))) return st;
    const Sched &s = p.sched[1][prec];
    const DevTables &D = p.dev[1][prec];
    hipStream_t hs = (hipStream_t)stream;
    const int64_t N = p.N;
    const DiagWork L = diag_layout(p, s, prec, batch);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, L.total, hs))) return st;
    void *W = at(sc.ptr, L.w);
    double *pp = (double *)at(sc.ptr, L.pp);
    // U = F u (the lattice DFT of the point values), as for the diagnostics
    ColArgs c = col_base(s, D, N);
    c.buf = W;
    c.buf_bs = s.L;
    c.in = u;
    c.in_bs = N;
    c.post_fwd = 1;
    c.chirp = s.bluestein ? 1 : 0;
    HIP_TRY(launch_col(prec, s, c, batch, hs), "projection transform");
    RowArgs r = row_base(s, D);
    r.buf = W;
    r.buf_bs = s.L;
    if (s.bluestein) {
        r.bhat = D.bhat;
        HIP_TRY(launch_row(prec, s, r, batch, hs), "projection transform");
        void *nat = at(sc.ptr, L.nat);
        ColArgs e = col_base(s, D, N);
        e.buf = W;
        e.buf_bs = s.L;
        e.pre_inv = 1;
        e.out = nat;
        e.out_bs = N;
        e.chirp = 1;
        HIP_TRY(launch_col(prec, s, e, batch, hs), "projection transform");  // unitary F u, key order
        HIP_TRY(launch_proj_sums(prec, nat, N, N, batch, 1.0 / std::sqrt((double)N), 0, s.L1, s.L2, ghat, N, pp,
                                 out, hs), "projection sums");
    } else {
        r.fft_only = 1;  // unnormalised F u at the row-pass positions
        HIP_TRY(launch_row(prec, s, r, batch, hs), "projection transform");
        HIP_TRY(launch_proj_sums(prec, W, s.L, N, batch, 1.0 / (double)N, transposed_layout(s) ? 1 : 0, s.L1, s.L2,
                                 ghat, N, pp, out, hs), "projection sums");
    }
    return LT_OK;
}

lt_status splitting_workspace_size(const lt_plan *p, lt_prec prec, int32_t batch, int32_t shared_v,
                                   int32_t order, size_t *bytes)
{
    if (!p || !bytes) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (batch < 0) return fail(LT_E_ARG, "batch must be >= 0");
    if (order != 2 && order != 4) return fail(LT_E_ARG, "order must be 2 or 4");
    double w[3];
    *bytes = composed_layout(*p, p->sched[1][prec], prec, batch, shared_v != 0, composition_weights(order, w)).total;
    return LT_OK;
}

lt_status splitting_times(int32_t order, int64_t steps, double t0, double dt, double *tau)
{
    if (order != 2 && order != 4) return fail(LT_E_ARG, "order must be 2 or 4");
    if (steps < 0) return fail(LT_E_ARG, "steps must be >= 0");
    if (!tau) return fail(LT_E_ARG, "tau is NULL");
    double w[3], c[4] = {0.0, 0.0, 0.0, 0.0};
    const int P = composition_weights(order, w);
    for (int i = 0; i < P; ++i) c[i + 1] = c[i] + w[i];
    for (int64_t k = 0; k < steps; ++k)
        for (int i = 0; i < P; ++i) tau[k * P + i] = t0 + ((double)k + c[i]) * dt;
    tau[steps * P] = t0 + (double)steps * dt;
    return LT_OK;
}

lt_status splitting_run(const lt_plan *cp, lt_prec prec, int32_t batch, const double *v, const double *v1,
                        int64_t v_stride, const double *f, void *u, double gamma, double dt, int64_t steps,
                        int32_t order, void *work, size_t work_bytes, void *stream)
{
    lt_status st = check_common(cp, prec, batch, gamma, dt, steps);
    if (st) return st;
    if (order != 2 && order != 4) return fail(LT_E_ARG, "order must be 2 or 4");
    lt_plan &p = *const_cast<lt_plan *>(cp);
    if (batch == 0 || steps == 0) return LT_OK;
    if (!v || !u) return fail(LT_E_ARG, "v and u must not be NULL");
    if (v1 && !f) return fail(LT_E_ARG, "a time-dependent field v1 needs its coefficients f");
    if (v_stride != 0 && v_stride < p.N) return fail(LT_E_ARG, "v_stride must be 0 or >= N");
    double w[3];
    const int P = composition_weights(order, w);
    const int64_t total = steps * P;  // substeps; f holds total + 1 values
    if (v1)
        for (int64_t j = 0; j <= total; ++j)
            if (!std::isfinite(f[j])) return fail(LT_E_ARG, "f must be finite");
    // the two-pass slot exists for every plan; chirp-z lattices use the
    // convolution form for every substep
    const Sched &s = p.sched[1][prec];
    if (s.bluestein && !conv_available(p, 1, s))
        return fail(LT_E_UNSUPPORTED, "no double-precision schedule for the convolution spectra");
    if ((st = ensure_device_tables(p, 1, prec, stream))) return st;
    if (s.bluestein && (st = ensure_device_tables(p, 1, LT_C128, stream))) return st;
    const DevTables &D = p.dev[1][prec];
    hipStream_t hs = (hipStream_t)stream;
    const ComposedWork L = composed_layout(p, s, prec, batch, v_stride == 0, P);
    Scratch sc;
    if ((st = get_work(sc, work, work_bytes, L.total, hs))) return st;
    const int64_t N = p.N;
    void *W = s.bluestein ? at(sc.ptr, L.w) : nullptr;
    Roles R[3];
    for (int i = 0; i < P; ++i) {
        const double dti = w[i] * dt;
        double *ktab = (double *)at(sc.ptr, L.ktab[i]);
        if ((st = make_ktab(p, s, ktab, gamma, dti, hs))) return st;
        void *conv = s.bluestein ? at(sc.ptr, L.conv[i]) : nullptr;
        if (conv && (st = conv_spectrum(p, 1, ktab, conv, at(sc.ptr, L.tmp), hs))) return st;
        // merged potential step after substep i: half phases of substeps i and i+1
        const double merged = (dti + w[(i + 1) % P] * dt) / (2.0 * gamma);
        // time-independent v: the merged phases as per-point tables
        void *ptab = !v1 ? at(sc.ptr, L.ptab[i]) : nullptr;
        if (ptab) HIP_TRY(launch_phase_table(prec, ptab, v, v_stride, v_stride ? batch : 1, N, merged, hs),
                          "potential table");
        R[i] = two_pass_roles(s, D, N, v, v_stride, u, W, dti / (2.0 * gamma), ktab, ptab);
        R[i].pot.phase = merged;
        R[i].first.chirp = 0;
        R[i].last.chirp = 0;
        if (conv) {
            R[i].row.bhat = (const double *)conv;
            if (prec == LT_C64) {
                void *cf = at(sc.ptr, L.conv_f[i]);
                HIP_TRY(launch_spectrum_f32(cf, conv, s.L, hs), "convolution spectrum (complex float)");
                R[i].row.bhat_f = (const float *)cf;
            }
        }
        if (v1) R[i].first.v2 = R[i].pot.v2 = R[i].last.v2 = v1;
    }
    // time-dependent field: the angle at substep boundary j carries f[j] v1
    ColArgs first = R[0].first;
    if (v1) first.phase2 = first.phase * f[0];
    HIP_TRY(launch_col(prec, s, first, batch, hs), "column pass");
    for (int64_t k = 0; k < total; ++k) {
        const Roles &r = R[k % P];
        HIP_TRY(launch_row(prec, s, r.row, batch, hs), "row pass");
        if (k == total - 1) break;
        ColArgs pot = r.pot;
        if (v1) pot.phase2 = pot.phase * f[k + 1];
        HIP_TRY(launch_col(prec, s, pot, batch, hs), "column pass (potential)");
    }
    ColArgs last = R[(total - 1) % P].last;
    if (v1) last.phase2 = last.phase * f[total];
    HIP_TRY(launch_col(prec, s, last, batch, hs), "column pass (last)");
    return LT_OK;
}

lt_status lattice_plan_set_kernels(lt_plan *p, lt_prec prec, int32_t col_variant, int32_t row_variant)
{
    if (!p) return fail(LT_E_ARG, "plan is NULL");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (col_variant < 0 || col_variant > 5 || row_variant < 0 || row_variant > 5)
        return fail(LT_E_ARG, "kernel variants are 0 to 5");
    std::lock_guard<std::mutex> lock(p->mu);
    for (int w = 0; w < 3; ++w) {
        Sched &s = p->sched[w][prec];
        if (s.passes < 2) continue;
        s.col_var = s.col_var_m = col_variant;
        s.row_var = s.row_var_m = row_variant;
    }
    return LT_OK;
}

lt_status lattice_plan_get_kernels_batch(const lt_plan *p, lt_prec prec, int32_t batch, int32_t *col_variant,
                                         int32_t *row_variant)
{
    if (!p || !col_variant || !row_variant) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (batch < 1) return fail(LT_E_ARG, "batch must be >= 1");
    const Sched &s = p->sched[2][prec].ok ? p->sched[2][prec] : p->sched[0][prec];
    *col_variant = col_variant_of(s, batch);
    *row_variant = row_variant_of(s, batch);
    return LT_OK;
}

lt_status lattice_plan_get_kernels(const lt_plan *p, lt_prec prec, int32_t *col_variant, int32_t *row_variant)
{
    if (!p || !col_variant || !row_variant) return fail(LT_E_ARG, "NULL argument");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    const Sched &s = p->sched[2][prec].ok ? p->sched[2][prec] : p->sched[0][prec];
    *col_variant = s.col_var;
    *row_variant = s.row_var;
    return LT_OK;
}

// Times the kernel variants of slot w's steady column and row passes on one
// state and on many; best_c / best_r receive the single-state [0] and
// many-state [1] choices.
static lt_status tune_slot(lt_plan *p, int w, lt_prec prec, int32_t reps, void *stream, int best_c[2], int best_r[2])
{
    lt_status st = ensure_device_tables(*p, w, prec, stream);
    if (st) return st;
    const Sched &s = p->sched[w][prec];
    const DevTables &D = p->dev[w][prec];
    hipStream_t hs = (hipStream_t)stream;
    // the many-state class is timed on about 2^22 points of states sharing v
    const int many = (int)std::max<int64_t>(2, ((int64_t(1) << 22) + s.L - 1) / s.L);
    void *buf = nullptr, *v = nullptr, *kt = nullptr, *pt = nullptr;
    const size_t ktn = (size_t)(p->max_s + 1);
    const size_t bytes = (size_t)many * s.L * esz(prec);
    HIP_TRY(hipMalloc(&buf, bytes), "autotune buffer");
    HIP_TRY(hipMalloc(&v, (size_t)p->N * sizeof(double)), "autotune buffer");
    HIP_TRY(hipMalloc(&kt, ktn * 16), "autotune buffer");
    HIP_TRY(hipMalloc(&pt, (size_t)p->N * 16), "autotune buffer");
    HIP_TRY(hipMemsetAsync(buf, 0, bytes, hs), "memset");
    HIP_TRY(hipMemsetAsync(v, 0, (size_t)p->N * sizeof(double), hs), "memset");
    HIP_TRY(launch_ktab((double *)kt, (int64_t)ktn, 0.0, 1.0, hs), "kinetic table");
    HIP_TRY(launch_phase_table(prec, pt, (const double *)v, 0, 1, p->N, 1e-3, hs), "potential table");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    ColArgs c = col_base(s, D, p->N);
    c.buf = buf;
    c.buf_bs = s.L;
    c.pre_inv = 1;
    c.post_fwd = 1;
    c.v = (const double *)v;
    c.phase = 1e-3;
    c.ptab = pt;
    c.ptab_bs = 0;
    RowArgs r = row_base(s, D);
    r.buf = buf;
    r.buf_bs = s.L;
    if (s.bluestein) r.bhat = D.bhat;
    else { r.s = D.s_row; r.ktab = (const double *)kt; }
    auto time_it = [&](bool col, int var, int batch, float &ms) -> lt_status {
        Sched t = s;
        t.col_var = t.col_var_m = t.row_var = t.row_var_m = var;
        for (int i = 0; i < reps + 2; ++i) {
            if (i == 2) HIP_TRY(hipEventRecord(e0, hs), "event");
            HIP_TRY(col ? launch_col(prec, t, c, batch, hs) : launch_row(prec, t, r, batch, hs),
                    "autotune launch");
        }
        HIP_TRY(hipEventRecord(e1, hs), "event");
        HIP_TRY(hipEventSynchronize(e1), "event");
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "event");
        return LT_OK;
    };
    // every candidate is timed in kTuneRounds interleaved rounds and its
    // fastest round counts, so that a transient slowdown (clock ramp, another
    // stream's work) does not decide the pick
    constexpr int kTuneRounds = 3;
    best_c[0] = best_c[1] = best_r[0] = best_r[1] = 0;
    for (int cls = 0; cls < 2 && !st; ++cls) {
        const int batch = cls ? many : 1;
        float tc[6], tr[6];
        for (int var = 0; var <= 5; ++var) tc[var] = tr[var] = 1e30f;
        for (int round = 0; round < kTuneRounds && !st; ++round) {
            for (int var = 0; var <= 5 && !st; ++var) {
                float ms = 0.f;
                if (var == 0 || fast_col_fits(prec, var, s.L1, s.L2, s.cols)) {
                    st = time_it(true, var, batch, ms);
                    if (!st) tc[var] = std::min(tc[var], ms);
                }
                if (!st && (var == 0 || fast_row_fits(prec, var, s.L1, s.L2, s.rows))) {
                    st = time_it(false, var, batch, ms);
                    if (!st) tr[var] = std::min(tr[var], ms);
                }
            }
        }
        for (int var = 1; var <= 5; ++var) {
            if (tc[var] < tc[best_c[cls]]) best_c[cls] = var;
            if (tr[var] < tr[best_r[cls]]) best_r[cls] = var;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(buf);
    hipFree(v);
    hipFree(kt);
    hipFree(pt);
    if (st) return st;
    return LT_OK;
}

lt_status lattice_plan_autotune(lt_plan *p, lt_prec prec, int32_t reps, void *stream)
{
    if (!p) return fail(LT_E_ARG, "plan is NULL");
    if (prec != LT_C64 && prec != LT_C128) return fail(LT_E_ARG, "bad precision");
    if (reps < 1) return fail(LT_E_ARG, "reps must be >= 1");
    if (!p->sched[0][prec].ok) return fail(LT_E_UNSUPPORTED, "no GPU schedule for this precision");
    if (p->sched[0][prec].passes != 2) return LT_OK;
    // slot 0 (and the adjoint's slot 1, the same schedule); slot 2 when the
    // plan has a swapped rank-2 schedule
    for (int w : {0, 2}) {
        if (w == 2 && !p->sched[2][prec].ok) continue;
        int bc[2], br[2];
        lt_status st = tune_slot(p, w, prec, reps, stream, bc, br);
        if (st) return st;
        std::lock_guard<std::mutex> lock(p->mu);
        for (int t = w; t <= (w == 0 ? 1 : 2); ++t) {
            Sched &x = p->sched[t][prec];
            if (x.passes < 2) continue;
            x.col_var = bc[0];
            x.row_var = br[0];
            x.col_var_m = bc[1];
            x.row_var_m = br[1];
        }
    }
    return LT_OK;
}

}  // extern "C"
