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
#include <thread>
#include <vector>

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
// Lexicographic enumeration of {h : lo < ||h||^2 <= hi} with h_1 in
// [x0, x1] (h_1 outermost), carrying the key's partial dot products
// sum_{j' < j} h_j' z_{i,j'} mod n_i down the recursion, so that a vector's
// key costs one multiply-add per level.
struct Shell {
    const lt_plan *p;
    int d, r;
    int64_t lo, hi;
    int32_t x0, x1;
    int32_t h[64];
    int64_t part[4][64];  // [component][level]
    template <class F> void walk(F &&f)
    {
        for (int i = 0; i < r; ++i) part[i][0] = 0;
        rec(0, 0, f);
    }
    template <class F> void rec(int j, int64_t used, F &f)
    {
        if (j == d) {
            if (used > lo) {
                int64_t chi = 0;
                for (int i = 0; i < r; ++i) {
                    int64_t xi = part[i][d] % p->n[i];
                    if (xi < 0) xi += p->n[i];
                    chi = chi * p->n[i] + xi;
                }
                f(h, used, chi);
            }
            return;
        }
        int64_t rem = hi - used;
        int32_t a = (int32_t)std::floor(std::sqrt((double)rem));
        while ((int64_t)(a + 1) * (a + 1) <= rem) ++a;
        while ((int64_t)a * a > rem) --a;
        int32_t from = -a, to = a;
        if (j == 0) {
            from = std::max(from, x0);
            to = std::min(to, x1);
        }
        for (int32_t x = from; x <= to; ++x) {
            h[j] = x;
            for (int i = 0; i < r; ++i)
                part[i][j + 1] = (part[i][j] + (int64_t)x * zr[i][j]) % p->n[i];
            rec(j + 1, used + (int64_t)x * x, f);
        }
    }
    int64_t zr[4][64];  // z_{i,j} mod n_i
};

// first-coordinate ranges for T threads over [-a, a], balanced by the
// volume of the remaining (d-1)-ball
std::vector<std::pair<int32_t, int32_t>> split_first(int d, int64_t hi, int T)
{
    int32_t a = (int32_t)std::floor(std::sqrt((double)hi));
    while ((int64_t)(a + 1) * (a + 1) <= hi) ++a;
    while ((int64_t)a * a > hi) --a;
    std::vector<double> w;
    double tot = 0;
    for (int32_t x = -a; x <= a; ++x) {
        const double rem = (double)(hi - (int64_t)x * x);
        const double wx = d > 1 ? std::pow(std::max(rem, 0.0) + 1.0, 0.5 * (d - 1)) : 1.0;
        w.push_back(wx);
        tot += wx;
    }
    std::vector<std::pair<int32_t, int32_t>> out;
    double acc = 0;
    int32_t start = -a;
    for (int32_t x = -a; x <= a; ++x) {
        acc += w[(size_t)(x + a)];
        if ((int)out.size() < T - 1 && acc >= tot * (double)(out.size() + 1) / T) {
            out.push_back({start, x});
            start = x + 1;
        }
    }
    if (start <= a) out.push_back({start, a});
    return out;
}
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
    if (d > 64 || p.r > 4) return fail(LT_E_UNSUPPORTED, "at most 64 dimensions and rank 4");
    Shell proto;
    proto.p = &p;
    proto.d = d;
    proto.r = p.r;
    for (int i = 0; i < p.r; ++i)
        for (int j = 0; j < d; ++j) {
            int64_t zz = p.Z[(size_t)i * d + j] % p.n[i];
            proto.zr[i][j] = zz < 0 ? zz + p.n[i] : zz;
        }
    const int T = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    while (count < N) {
        // the vectors of the range (lo, hi], placed in (norm, lex) order: each
        // thread walks a contiguous range of first coordinates (so its
        // vectors of one norm are a contiguous lex range), counts them per
        // norm, then writes them at offsets ordered by (norm, thread)
        const int64_t base = lo < 0 ? 0 : lo + 1;
        const size_t nn = (size_t)(hi - base + 1);
        const auto parts = split_first(d, hi, T);
        const int P = (int)parts.size();
        std::vector<std::vector<int64_t>> cnt((size_t)P, std::vector<int64_t>(nn, 0));
        std::vector<int32_t> amax_t((size_t)P, 0);
        auto run = [&](auto &&body) {
            std::vector<std::thread> th;
            for (int t = 0; t < P; ++t) th.emplace_back([&, t]() { body(t); });
            for (auto &x : th) x.join();
        };
        run([&](int t) {
            Shell sh = proto;
            sh.lo = lo;
            sh.hi = hi;
            sh.x0 = parts[(size_t)t].first;
            sh.x1 = parts[(size_t)t].second;
            int64_t *c = cnt[(size_t)t].data();
            int32_t am = 0;
            sh.walk([&](const int32_t *h, int64_t sn, int64_t) {
                ++c[sn - base];
                for (int j = 0; j < d; ++j) am = std::max(am, std::abs(h[j]));
            });
            amax_t[(size_t)t] = am;
        });
        int64_t total = 0;
        int32_t amax = 0;
        std::vector<std::vector<int64_t>> off((size_t)P, std::vector<int64_t>(nn, 0));
        std::vector<int64_t> norm_start(nn + 1, 0);
        for (size_t k = 0; k < nn; ++k) {
            norm_start[k] = total;
            for (int t = 0; t < P; ++t) {
                off[(size_t)t][k] = total;
                total += cnt[(size_t)t][k];
            }
        }
        norm_start[nn] = total;
        for (int t = 0; t < P; ++t) amax = std::max(amax, amax_t[(size_t)t]);
        enumerated += total;
        if (enumerated > budget)
            return fail(LT_E_UNSUPPORTED,
                        "minimal-l2 completion needs more than " + std::to_string(budget) +
                            " frequency vectors (" + std::to_string(N - count) +
                            " keys still uncovered at squared radius " + std::to_string(lo < 0 ? 0 : lo) +
                            "): the generating vector has short dual vectors; choose a better lattice");
        const bool narrow = amax <= 127;
        std::vector<int8_t> h8(narrow ? (size_t)total * d : 0);
        std::vector<int32_t> h32(narrow ? 0 : (size_t)total * d);
        std::vector<int64_t> keys((size_t)total);
        run([&](int t) {
            Shell sh = proto;
            sh.lo = lo;
            sh.hi = hi;
            sh.x0 = parts[(size_t)t].first;
            sh.x1 = parts[(size_t)t].second;
            std::vector<int64_t> &o = off[(size_t)t];
            sh.walk([&](const int32_t *h, int64_t sn, int64_t chi) {
                const int64_t at = o[(size_t)(sn - base)]++;
                keys[(size_t)at] = chi;
                for (int j = 0; j < d; ++j) {
                    if (narrow) h8[(size_t)at * d + j] = (int8_t)h[j];
                    else h32[(size_t)at * d + j] = h[j];
                }
            });
        });
        // first vector in (norm, lex) order wins each key
        for (size_t k = 0; k < nn && count < N; ++k) {
            const int64_t sn = base + (int64_t)k;
            for (int64_t at = norm_start[k]; at < norm_start[k + 1] && count < N; ++at) {
                const int64_t chi = keys[(size_t)at];
                if (owned[(size_t)chi]) continue;
                owned[(size_t)chi] = 1;
                p.s_of_key[(size_t)chi] = sn;
                int32_t *dst = &p.h_of_key[(size_t)chi * d];
                for (int j = 0; j < d; ++j) dst[j] = narrow ? h8[(size_t)at * d + j] : h32[(size_t)at * d + j];
                ++count;
            }
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
