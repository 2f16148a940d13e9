// Host planner: lattice validation, keys, the full anti-aliasing set and the
// GPU transform schedule.
//
// Index set (Def. 2, Thm. 1, Lemma 4): the user set H owns its keys; every
// other key receives its minimal-l2 representative using the construction
// of Sec. 3.1 -- enumerate all h with ||h||^2 <= R^2, visit them sorted by
// norm (ties: lexicographic, h_1 first), and give each not-yet-owned key to
// the first vector that reaches it.  If the ball does not reach every key,
// the next shell is visited, so the visiting order stays (norm, lex).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "lt_internal.h"

namespace lt {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

lt_status fail(lt_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

static int64_t gcd64(int64_t a, int64_t b)
{
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a;
}

static inline int64_t key_of(const lt_plan &p, const int32_t *h)
{
    int64_t chi = 0;
    for (int i = 0; i < p.r; ++i) {
        __int128 dot = 0;
        const int64_t *z = p.Z.data() + (size_t)i * p.d;
        for (int j = 0; j < p.d; ++j) dot += (__int128)h[j] * z[j];
        int64_t xi = (int64_t)(dot % p.n[i]);
        if (xi < 0) xi += p.n[i];
        chi = chi * p.n[i] + xi;
    }
    return chi;
}

// Distinct points <=> only k = 0 is mapped to the origin (the point map is a
// group homomorphism from Z_{n_1} + ... + Z_{n_r} to the torus).
static bool points_distinct(const lt_plan &p)
{
    if (p.r == 1) {
        int64_t g = p.N;
        for (int j = 0; j < p.d; ++j) g = gcd64(g, p.Z[j]);
        return g == 1;
    }
    std::vector<int64_t> k(p.r);
    for (int64_t kappa = 1; kappa < p.N; ++kappa) {
        int64_t rem = kappa;
        for (int i = p.r - 1; i >= 0; --i) { k[i] = rem % p.n[i]; rem /= p.n[i]; }
        bool zero = true;
        for (int j = 0; j < p.d && zero; ++j) {
            __int128 acc = 0;
            for (int i = 0; i < p.r; ++i)
                acc += (__int128)p.Z[(size_t)i * p.d + j] * k[i] * (p.N / p.n[i]);
            if (acc % p.N != 0) zero = false;
        }
        if (zero) return false;
    }
    return true;
}

namespace {
// Lexicographic enumeration of {h : lo < ||h||^2 <= hi}, h_1 outermost.
struct Shell {
    int d;
    int64_t lo, hi;
    std::vector<int32_t> h;
    int64_t limit = INT64_MAX, seen = 0;  // the walk stops after `limit` vectors
    template <class F> void walk(F &&f) { h.assign(d, 0); seen = 0; rec(0, 0, f); }
    template <class F> void rec(int j, int64_t used, F &f)
    {
        if (seen >= limit) return;
        if (j == d) {
            if (used > lo) {
                f(h.data(), used);
                ++seen;
            }
            return;
        }
        int64_t rem = hi - used;
        int32_t a = (int32_t)std::floor(std::sqrt((double)rem));
        while ((int64_t)(a + 1) * (a + 1) <= rem) ++a;
        while ((int64_t)a * a > rem) --a;
        for (int32_t x = -a; x <= a; ++x) {
            h[j] = x;
            rec(j + 1, used + (int64_t)x * x, f);
        }
    }
};
}  // namespace

lt_status plan_index_set(lt_plan &p)
{
    const int64_t N = p.N;
    const int d = p.d;
    if (!points_distinct(p))
        return fail(LT_E_INCOMPLETE, "lattice points are not distinct, so not every key is reachable");

    std::vector<uint8_t> owned((size_t)N, 0);
    p.s_of_key.assign((size_t)N, -1);
    p.h_of_key.assign((size_t)N * d, 0);
    const int64_t nh = (int64_t)p.H.size() / d;
    p.key_of_h.resize((size_t)nh);
    int64_t count = 0;
    for (int64_t t = 0; t < nh; ++t) {
        const int32_t *h = p.H.data() + (size_t)t * d;
        int64_t chi = key_of(p, h);
        p.key_of_h[(size_t)t] = chi;
        if (owned[(size_t)chi])
            return fail(LT_E_NOT_INJECTIVE, "index set rows " + std::to_string(t) +
                        " and an earlier row share key " + std::to_string(chi));
        owned[(size_t)chi] = 1;
        int64_t s = 0;
        for (int j = 0; j < d; ++j) s += (int64_t)h[j] * h[j];
        p.s_of_key[(size_t)chi] = s;
        std::memcpy(&p.h_of_key[(size_t)chi * d], h, (size_t)d * sizeof(int32_t));
        ++count;
    }
    p.n_index = nh;
    p.n_completed = N - nh;
    if (!p.complete && nh > 0 && count < N)
        return fail(LT_E_INCOMPLETE, "the index set owns " + std::to_string(count) + " of " + std::to_string(N) +
                    " keys; plan with complete = 1 to give the others their minimal-l2 representatives");

    // initial radius: a ball holding about N lattice vectors
    double lg = std::lgamma(0.5 * d + 1.0) + std::log((double)N) - 0.5 * d * std::log(M_PI);
    int64_t hi = (int64_t)std::floor(std::exp(2.0 * lg / d));
    if (hi < 1) hi = 1;
    int64_t lo = -1;
    // A lattice whose dual has short vectors leaves keys uncovered until the
    // ball is far larger than N; bound the enumeration instead of exhausting
    // host memory.
    const int64_t budget = std::max<int64_t>(int64_t(1) << 26, 64 * N);
    int64_t enumerated = 0;
    while (count < N) {
        // count the shell per norm, then place vectors in (norm, lex) order
        Shell sh{d, lo, hi, {}};
        sh.limit = budget - enumerated + 1;
        std::vector<int64_t> per((size_t)(hi - (lo < 0 ? 0 : lo) + 2), 0);
        const int64_t base = lo < 0 ? 0 : lo + 1;
        int64_t total = 0;
        int32_t amax = 0;
        sh.walk([&](const int32_t *h, int64_t s) {
            ++per[(size_t)(s - base)];
            ++total;
            for (int j = 0; j < d; ++j) amax = std::max(amax, std::abs(h[j]));
        });
        enumerated += total;
        if (enumerated > budget)
            return fail(LT_E_UNSUPPORTED,
                        "minimal-l2 completion needs more than " + std::to_string(budget) +
                            " frequency vectors (" + std::to_string(N - count) +
                            " keys still uncovered at squared radius " + std::to_string(lo < 0 ? 0 : lo) +
                            "): the generating vector has short dual vectors; choose a better lattice");
        std::vector<int64_t> off(per.size() + 1, 0);
        for (size_t t = 0; t < per.size(); ++t) off[t + 1] = off[t] + per[t];
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        const bool narrow = amax <= 127;
        std::vector<int8_t> h8(narrow ? (size_t)total * d : 0);
        std::vector<int32_t> h32(narrow ? 0 : (size_t)total * d);
        std::vector<int64_t> snorm((size_t)total);
        sh.walk([&](const int32_t *h, int64_t s) {
            int64_t at = fill[(size_t)(s - base)]++;
            snorm[(size_t)at] = s;
            for (int j = 0; j < d; ++j) {
                if (narrow) h8[(size_t)at * d + j] = (int8_t)h[j];
                else h32[(size_t)at * d + j] = h[j];
            }
        });
        std::vector<int32_t> hv(d);
        for (int64_t at = 0; at < total && count < N; ++at) {
            for (int j = 0; j < d; ++j)
                hv[j] = narrow ? h8[(size_t)at * d + j] : h32[(size_t)at * d + j];
            int64_t chi = key_of(p, hv.data());
            if (owned[(size_t)chi]) continue;
            owned[(size_t)chi] = 1;
            p.s_of_key[(size_t)chi] = snorm[(size_t)at];
            std::memcpy(&p.h_of_key[(size_t)chi * d], hv.data(), (size_t)d * sizeof(int32_t));
            ++count;
        }
        lo = hi;
        hi = hi + hi / 3 + 1;
    }
    p.max_s = 0;
    for (int64_t t = 0; t < N; ++t) p.max_s = std::max(p.max_s, p.s_of_key[(size_t)t]);
    return LT_OK;
}

// ---------------------------------------------------------------- schedules
bool factor_radices(int64_t L, Radices &out, int max_log2)
{
    // Power-of-two part in as few stages as possible (radix <= 2^max_log2),
    // spread evenly (512 = 8*8*8 rather than 16*16*2); then the odd radices
    // 7, 5, 3.
    out.L = (int)L;
    out.n = 0;
    if (L < 1) return false;
    int64_t m = L;
    int e = 0;
    while (m % 2 == 0) { m /= 2; ++e; }
    std::vector<int> st;
    if (e > 0) {
        int k = (e + max_log2 - 1) / max_log2;
        for (int i = 0; i < k; ++i) st.push_back(1 << (e / k + (i < e % k ? 1 : 0)));
    }
    for (int f : {7, 5, 3})
        while (m % f == 0) { st.push_back(f); m /= f; }
    if (m != 1 || (int)st.size() > kMaxStages) return false;
    for (int R : st) out.r[out.n++] = R;
    return true;
}

static bool is_smooth7(int64_t x)
{
    if (x < 1) return false;
    for (int f : {2, 3, 5, 7})
        while (x % f == 0) x /= f;
    return x == 1;
}

int64_t smooth7_at_least(int64_t x)
{
    int64_t best = -1;
    for (int64_t a = 1; a < 4 * x; a *= 2)
        for (int64_t b = a; b < 4 * x; b *= 3)
            for (int64_t c = b; c < 4 * x; c *= 5)
                for (int64_t e = c; e < 4 * x; e *= 7)
                    if (e >= x && (best < 0 || e < best)) best = e;
    return best;
}

// Pick the column length L1 (a divisor of L) closest to the target, with
// L2 = L / L1 fitting one workgroup tile.
static bool split_two_pass(int64_t L, int64_t tile, int &L1, int &L2)
{
    int64_t best = -1;
    double target = std::min<double>(std::sqrt((double)L), 512.0);
    for (int64_t a = 2; a <= tile && a < L; ++a) {
        if (L % a) continue;
        int64_t b = L / a;
        if (b > tile) continue;
        if (!is_smooth7(a) || !is_smooth7(b)) continue;
        if (best < 0 || std::fabs(std::log((double)a / target)) <
                            std::fabs(std::log((double)best / target)))
            best = a;
    }
    if (best < 0) {
        if (L > tile) return false;
        best = 1;  // degenerate split for tiny L: one column pass of length 1
    }
    L1 = (int)best;
    L2 = (int)(L / best);
    return true;
}

Sched make_schedule(const lt_plan &p, int prec, bool force_two_pass)
{
    Sched s;
    const int64_t tile = kTileElems;  // complex elements per workgroup tile
    s.ept = (int)(tile / kThreads);
    // general kernels: radix 16 butterflies in double need too many registers
    const int mr = prec == LT_C128 ? 3 : 4;
    if (p.r > 2) return s;
    if (p.r == 2) {
        if (!is_smooth7(p.n[0]) || !is_smooth7(p.n[1])) return s;
        s.rank2 = true;
        s.L = p.N;
        s.L1 = (int)p.n[0];
        s.L2 = (int)p.n[1];
        if (p.n[0] > tile || p.n[1] > tile) return s;
        if (!factor_radices(p.n[0], s.ra, mr) || !factor_radices(p.n[1], s.rb, mr)) return s;
        if (p.N <= tile && !force_two_pass) {
            s.passes = 1;
        } else {
            s.passes = 2;
            s.cols = (int)std::max<int64_t>(1, std::min<int64_t>(tile / s.L1, s.L2));
            s.rows = (int)std::max<int64_t>(1, std::min<int64_t>(tile / s.L2, s.L1));
        }
        s.ok = true;
        return s;
    }
    // Smooth N: the DFT of length N itself -- unless N is not a power of two
    // and needs two passes: its factors 3, 5, 7 only fit the general passes
    // (runtime radices), so it takes the chirp-z convolution of power-of-two
    // length >= 2N - 1 like a prime, whose passes are register-staged (about
    // 3x cheaper per element, and with more workgroups), while that length
    // has a two-pass split.
    bool direct = is_smooth7(p.N);
    if (direct && (p.N & (p.N - 1)) != 0 && p.N > tile) {
        int64_t q = 1;
        while (q < 2 * p.N - 1) q <<= 1;
        if (q <= tile * kWideRow) direct = false;
    }
    if (direct) {
        s.L = p.N;
    } else {
        // chirp-z length: any L >= 2N - 1 works.  One workgroup's tile: the
        // smallest 7-smooth length; two passes: a power of two, whose factors
        // the register-staged passes cover (up to 2x the 7-smooth length, at
        // a fraction of the cost per element of the general passes)
        s.bluestein = true;
        s.L = smooth7_at_least(2 * p.N - 1);
        if (s.L > tile || force_two_pass) {
            int64_t q = 1;
            while (q < 2 * p.N - 1) q <<= 1;
            if (q <= tile * kWideRow) s.L = q;
        }
    }
    // power-of-two transforms of 2^24 points or more: three levels, so that
    // no pass holds a 4096-point column (one column per tile, one cache line
    // per element); L1 = 512 columns (8 per tile), an inner level of 64, rows
    // of L / 32768 (512 or 1024 points)
    if (!s.bluestein && !force_two_pass && (s.L & (s.L - 1)) == 0 && s.L >= ((int64_t)1 << 24) &&
        s.L <= ((int64_t)1 << 25)) {
        s.L1 = 512;
        s.L2 = 64;
        s.L3 = (int)(s.L / (512 * 64));
        if (!factor_radices(s.L1, s.ra, mr) || !factor_radices(s.L2, s.rc, mr) || !factor_radices(s.L3, s.rb, mr))
            return s;
        s.passes = 3;
        s.cols = (int)(tile / s.L1);
        s.cols2 = (int)(tile / s.L2);
        s.rows = (int)(tile / s.L3);
        s.ok = true;
        return s;
    }
    if (s.L <= tile && !force_two_pass) {
        s.passes = 1;
        s.L1 = (int)s.L;
        s.L2 = 1;
        if (!factor_radices(s.L, s.ra, mr)) return s;
        s.rb = s.ra;
        s.ok = true;
        return s;
    }
    if (!split_two_pass(s.L, tile, s.L1, s.L2)) {
        // above tile^2 points: rows of kWideRow points, one per workgroup
        // (columns of at most one tile)
        if (s.L % kWideRow || s.L / kWideRow > tile || !is_smooth7(s.L / kWideRow)) return s;
        s.L1 = (int)(s.L / kWideRow);
        s.L2 = (int)kWideRow;
    }
    if (!factor_radices(s.L1, s.ra, mr) || !factor_radices(s.L2, s.rb, mr)) return s;
    s.passes = 2;
    s.cols = (int)std::max<int64_t>(1, std::min<int64_t>(tile / s.L1, s.L2));
    s.rows = (int)std::max<int64_t>(1, std::min<int64_t>(tile / s.L2, s.L1));
    s.ok = true;
    return s;
}

}  // namespace lt

extern "C" const char *lt_last_error(void) { return lt::g_err.c_str(); }
