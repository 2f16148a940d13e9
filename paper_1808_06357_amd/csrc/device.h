// Device-side building blocks shared by the HIP kernels: complex arithmetic,
// accurate constant / twiddle multiplies, FP64 phases and the small DFTs.
//
// Accuracy rule for the complex64 path: every multiplication by a *constant*
// (butterfly constants, twiddles, phases, the chirp-z kernel spectrum) is
// carried out beyond FP32 precision -- constants are split into hi + lo float
// pairs or applied in double -- so the only FP32 errors left are the
// data-dependent roundings of the results.  A constant rounded to FP32 would
// repeat the same error in every time step and accumulate linearly over the
// run (a 1-ulp magnitude bias of a butterfly constant alone drifts the norm by
// ~1e-7 per step).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lt_internal.h"

namespace lt {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> mul_negi(cx<T> a) { return {a.y, -a.x}; }   // (-i) a
template <typename T>
__device__ __forceinline__ cx<T> scal(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------- twiddle tables
// Table element type: complex double for complex128 runs; a hi + lo pair of
// complex floats (hi = fl(w), lo = fl(w - hi)) for complex64 runs.
template <typename T>
struct Tw;
template <>
struct Tw<double> {
    cx<double> w;
};
template <>
struct Tw<float> {
    cx<float> hi, lo;
};

__device__ __forceinline__ cx<double> twmul(cx<double> a, const Tw<double> &t) { return cmul(a, t.w); }
__device__ __forceinline__ cx<float> twmul(cx<float> a, const Tw<float> &t)
{
    // a * (hi + lo): the lo part is folded in with FMAs before rounding
    const float rl = a.x * t.lo.x - a.y * t.lo.y;
    const float il = a.x * t.lo.y + a.y * t.lo.x;
    return {__fmaf_rn(a.x, t.hi.x, __fmaf_rn(-a.y, t.hi.y, rl)),
            __fmaf_rn(a.x, t.hi.y, __fmaf_rn(a.y, t.hi.x, il))};
}

// a * (wr + i wi) for a double-precision complex w known at run time
__device__ __forceinline__ cx<double> cmul_d(cx<double> a, double wr, double wi)
{
    return {a.x * wr - a.y * wi, a.x * wi + a.y * wr};
}
__device__ __forceinline__ cx<float> cmul_d(cx<float> a, double wr, double wi)
{
    const double x = a.x, y = a.y;
    return {(float)(x * wr - y * wi), (float)(x * wi + y * wr)};
}

// x * r for a compile-time constant r: exact split for float
__device__ __forceinline__ double mulc(double x, double r) { return x * r; }
__device__ __forceinline__ float mulc(float x, double r)
{
    const float hi = (float)r;
    const float lo = (float)(r - (double)hi);
    return __fmaf_rn(x, hi, x * lo);
}
// a * (wr + i wi), compile-time constant
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, double wr, double wi)
{
    return {mulc(a.x, wr) - mulc(a.y, wi), mulc(a.x, wi) + mulc(a.y, wr)};
}

// ---------------------------------------------------------------- FP64 phases
// exp(-i a) for a double angle: reduce a mod 2 pi in double (Cody-Waite split
// of 2 pi), then sincos in double.
__device__ __forceinline__ void expm_i(double a, double &c, double &s)
{
    const double inv2pi = 0.15915494309189533577;
    const double twopi_hi = 6.28318530717958623200;     // 2 pi rounded to double
    const double twopi_lo = 2.44929359829470635445e-16;  // 2 pi - twopi_hi
    const double q = rint(a * inv2pi);
    double r = __fma_rn(-q, twopi_hi, a);
    r = __fma_rn(-q, twopi_lo, r);
    double sn, cs;
    sincos(r, &sn, &cs);
    c = cs;
    s = -sn;
}

// table entry as a double-precision complex (hi + lo for the float tables)
__device__ __forceinline__ cx<double> tw_d(const Tw<double> &t) { return t.w; }
__device__ __forceinline__ cx<double> tw_d(const Tw<float> &t)
{
    return {(double)t.hi.x + (double)t.lo.x, (double)t.hi.y + (double)t.lo.y};
}

// w^r for r = 0..R-1 in double by a balanced product tree
// (w^r = w^(r/2) w^(r - r/2)): at most log2(R) rounding steps deep
template <int R>
__device__ __forceinline__ void powers(double wr, double wi, double (&pr)[R], double (&pi)[R])
{
    pr[0] = 1.0;
    pi[0] = 0.0;
    if constexpr (R > 1) {
        pr[1] = wr;
        pi[1] = wi;
    }
#pragma unroll
    for (int r = 2; r < R; ++r) {
        const int a = r / 2, b = r - r / 2;
        pr[r] = pr[a] * pr[b] - pi[a] * pi[b];
        pi[r] = pr[a] * pi[b] + pi[a] * pr[b];
    }
}

// member k of a batch list with start[k] <= bid < start[k+1] (binary search)
__device__ __forceinline__ int find_member(const int *start, int n, int bid)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (start[mid] <= bid) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Work item of block b in a grid of n blocks (n a multiple of 8).  Blocks are
// dealt round-robin to the 8 XCDs (block b to XCD b mod 8), each with its own
// L2; this hands every XCD a contiguous range of work items, so that
// neighbouring column tiles, which share cache lines, meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int n) { return (b & 7) * (n >> 3) + (b >> 3); }

// floor(x / d) by a double reciprocal, for 0 <= x < 2^50 and d >= 1: the
// quotient (x + 1/2) / d lies at least 1/(2d) from an integer, far beyond the
// relative error 2^-52 of the two roundings
struct FDiv {
    int d;
    double r;
};
__device__ __forceinline__ FDiv fdiv_make(int d) { return {d, 1.0 / (double)d}; }
__device__ __forceinline__ int fdiv(int x, const FDiv &f) { return (int)(((double)x + 0.5) * f.r); }
__device__ __forceinline__ int64_t fdiv64(int64_t x, const FDiv &f) { return (int64_t)(((double)x + 0.5) * f.r); }

// Sum of two per-thread doubles over a workgroup of NT threads (NT a
// multiple of 64), in a fixed order: a butterfly across each wave, then the
// waves in order.  The totals land in thread 0; every thread must call it.
template <int NT>
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    __shared__ double red[2][NT / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = a;
        red[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = red[0][0];
        b = red[1][0];
#pragma unroll
        for (int i = 1; i < NT / 64; ++i) {
            a += red[0][i];
            b += red[1][i];
        }
    }
    __syncthreads();
}

// chirp c_n = exp(-pi i (n^2 mod 2N) / N), exact integer reduction
__device__ __forceinline__ void chirp(int64_t n, int64_t N, double &c, double &s)
{
    // n < N < 2^31, so n^2 < 2^62 fits in 64 bits
    const int64_t q = (int64_t)(((uint64_t)n * (uint64_t)n) % (uint64_t)(2 * N));
    double sn, cs;
    sincospi((double)q / (double)N, &sn, &cs);
    c = cs;
    s = -sn;
}

// ---------------------------------------------------------------- butterflies
// Forward small DFTs, X_k = sum_j v_j exp(-2 pi i j k / R), natural order.
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <typename T>
struct Dft<T, 4> {
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        cx<T> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = mul_negi(v[1] - v[3]);
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + d;
        v[3] = b - d;
    }
};

constexpr double kSqrtHalf = 0.70710678118654752440084436210484904;

template <typename T>
struct Dft<T, 8> {
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, 4>::run(e);
        Dft<T, 4>::run(o);
        o[1] = {mulc(o[1].x + o[1].y, kSqrtHalf), mulc(o[1].y - o[1].x, kSqrtHalf)};
        o[2] = mul_negi(o[2]);
        o[3] = {mulc(o[3].y - o[3].x, kSqrtHalf), -mulc(o[3].x + o[3].y, kSqrtHalf)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = e[k] + o[k];
            v[k + 4] = e[k] - o[k];
        }
    }
};

// cos(2 pi m / 16)
__device__ __forceinline__ constexpr double c16(int m)
{
    constexpr double t[16] = {1.0,
                              0.92387953251128675612818318939678829,
                              0.70710678118654752440084436210484904,
                              0.38268343236508977172845998403039887,
                              0.0,
                              -0.38268343236508977172845998403039887,
                              -0.70710678118654752440084436210484904,
                              -0.92387953251128675612818318939678829,
                              -1.0,
                              -0.92387953251128675612818318939678829,
                              -0.70710678118654752440084436210484904,
                              -0.38268343236508977172845998403039887,
                              0.0,
                              0.38268343236508977172845998403039887,
                              0.70710678118654752440084436210484904,
                              0.92387953251128675612818318939678829};
    return t[m & 15];
}
__device__ __forceinline__ constexpr double s16(int m) { return c16((m + 12) & 15); }  // sin(2 pi m/16)

template <typename T>
struct Dft<T, 16> {
    // 16 = 4 x 4: radix-4 DFTs over j2 (stride 4), twiddle W16^{j1 k2},
    // radix-4 DFTs over j1.
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        cx<T> a[4][4];
#pragma unroll
        for (int j1 = 0; j1 < 4; ++j1) {
#pragma unroll
            for (int j2 = 0; j2 < 4; ++j2) a[j1][j2] = v[j1 + 4 * j2];
            Dft<T, 4>::run(a[j1]);
#pragma unroll
            for (int k2 = 1; k2 < 4; ++k2) {
                const int m = j1 * k2;
                if (m == 0) continue;
                if (m == 4) { a[j1][k2] = mul_negi(a[j1][k2]); continue; }
                a[j1][k2] = cmulc(a[j1][k2], c16(m), -s16(m));
            }
        }
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            cx<T> b[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
            Dft<T, 4>::run(b);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = b[k1];
        }
    }
};

// odd radices: X_k = v_0 + sum_{j=1}^{(R-1)/2} [(v_j + v_{R-j}) cos(2 pi jk/R)
//                                               - i (v_j - v_{R-j}) sin(2 pi jk/R)]
template <int R>
__device__ __forceinline__ constexpr double cosr(int m);
template <int R>
__device__ __forceinline__ constexpr double sinr(int m);
template <>
__device__ __forceinline__ constexpr double cosr<3>(int m)
{
    constexpr double t[3] = {1.0, -0.5, -0.5};
    return t[m];
}
template <>
__device__ __forceinline__ constexpr double sinr<3>(int m)
{
    constexpr double t[3] = {0.0, 0.86602540378443864676372317075293618,
                             -0.86602540378443864676372317075293618};
    return t[m];
}
template <>
__device__ __forceinline__ constexpr double cosr<5>(int m)
{
    constexpr double t[5] = {1.0, 0.30901699437494742410229341718281906,
                             -0.80901699437494742410229341718281906,
                             -0.80901699437494742410229341718281906,
                             0.30901699437494742410229341718281906};
    return t[m];
}
template <>
__device__ __forceinline__ constexpr double sinr<5>(int m)
{
    constexpr double t[5] = {0.0, 0.95105651629515357211643933337938214,
                             0.58778525229247312916870595463907277,
                             -0.58778525229247312916870595463907277,
                             -0.95105651629515357211643933337938214};
    return t[m];
}
template <>
__device__ __forceinline__ constexpr double cosr<7>(int m)
{
    constexpr double t[7] = {1.0,
                             0.62348980185873353052500488400423981,
                             -0.22252093395631440428890256449679476,
                             -0.90096886790241912623610231950744505,
                             -0.90096886790241912623610231950744505,
                             -0.22252093395631440428890256449679476,
                             0.62348980185873353052500488400423981};
    return t[m];
}
template <>
__device__ __forceinline__ constexpr double sinr<7>(int m)
{
    constexpr double t[7] = {0.0,
                             0.78183148246802980870844452667405775,
                             0.97492791218182360701813168299393122,
                             0.43388373911755812047576833284835875,
                             -0.43388373911755812047576833284835875,
                             -0.97492791218182360701813168299393122,
                             -0.78183148246802980870844452667405775};
    return t[m];
}

template <typename T, int R>
struct DftOdd {
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        constexpr int H = (R - 1) / 2;
        cx<T> a[H], b[H];
        cx<T> out[R];
        cx<T> sum = v[0];
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            a[j - 1] = v[j] + v[R - j];
            b[j - 1] = v[j] - v[R - j];
            sum = sum + a[j - 1];
        }
        out[0] = sum;
#pragma unroll
        for (int k = 1; k < R; ++k) {
            T re = v[0].x, im = v[0].y;
#pragma unroll
            for (int j = 1; j <= H; ++j) {
                const int m = (j * k) % R;
                re += mulc(a[j - 1].x, cosr<R>(m)) + mulc(b[j - 1].y, sinr<R>(m));
                im += mulc(a[j - 1].y, cosr<R>(m)) - mulc(b[j - 1].x, sinr<R>(m));
            }
            out[k] = {re, im};
        }
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = out[k];
    }
};
template <typename T>
struct Dft<T, 3> : DftOdd<T, 3> {};
template <typename T>
struct Dft<T, 5> : DftOdd<T, 5> {};
template <typename T>
struct Dft<T, 7> : DftOdd<T, 7> {};

// four-step twiddle W_L^{n2 k1} (L = L1 L2) from two double tables, applied in double
template <typename T>
__device__ __forceinline__ cx<T> tw4mul(cx<T> x, int n2, int k1, const FDiv &L2d, const double *hi,
                                        const double *lo)
{
    const int64_t q = (int64_t)n2 * k1;
    const int qa = (int)fdiv64(q, L2d);
    const int qb = (int)(q - (int64_t)qa * L2d.d);
    const double ax = hi[2 * qa], ay = hi[2 * qa + 1], bx = lo[2 * qb], by = lo[2 * qb + 1];
    return cmul_d(x, ax * bx - ay * by, ax * by + ay * bx);
}

template <typename T>
__device__ __forceinline__ cx<T> tw4mul(cx<T> x, int n2, int k1, int L2, const double *hi, const double *lo)
{
    const int64_t q = (int64_t)n2 * k1;
    int qa, qb;
    if ((L2 & (L2 - 1)) == 0) {
        const int sh = __builtin_ctz((unsigned)L2);
        qa = (int)(q >> sh);
        qb = (int)(q & (L2 - 1));
    } else {
        qa = (int)(q / L2);
        qb = (int)(q - (int64_t)qa * L2);
    }
    const double ax = hi[2 * qa], ay = hi[2 * qa + 1], bx = lo[2 * qb], by = lo[2 * qb + 1];
    return cmul_d(x, ax * bx - ay * by, ax * by + ay * bx);
}

// x * exp(-i a) with the phase evaluated and applied in double
template <typename T>
__device__ __forceinline__ cx<T> mul_expm_i(cx<T> x, double a)
{
    double c, s;
    expm_i(a, c, s);
    return cmul_d(x, c, s);
}


// point-domain multiplier of a column pass (see ColArgs)
template <typename T>
__device__ __forceinline__ cx<T> col_mid(cx<T> x, const ColArgs &a, const double *vb, const double *vb2,
                                         int64_t n)
{
    const bool any = vb || a.ktab || a.chirp || a.scale != 1.0;
    if (!any) return x;
    double c = 1.0, s = 0.0;
    if (vb) expm_i(vb2 ? a.phase * vb[n] + a.phase2 * vb2[n] : a.phase * vb[n], c, s);
    if (a.ktab) {
        const int m = a.s[n];
        const double kr = a.ktab[2 * m], ki = a.ktab[2 * m + 1];
        const double r = c * kr - s * ki, i = c * ki + s * kr;
        c = r;
        s = i;
    }
    if (a.chirp) {
        double cc, cs;
        chirp(n, a.Nchirp, cc, cs);
        if (a.chirp < 0) cs = -cs;
        const double r = c * cc - s * cs, i = c * cs + s * cc;
        c = r;
        s = i;
    }
    return cmul_d(x, c * a.scale, s * a.scale);
}

// checkpoint store of the lattice value u = x exp(-i ck_phase v) [conj(c_n)]
template <typename T>
__device__ __forceinline__ void col_checkpoint(cx<T> x, const ColArgs &a, int64_t b, int64_t n)
{
    double c, sn;
    expm_i(a.ck_phase * a.ck_v[b * a.v_bs + n], c, sn);
    if (a.ck_chirp) {
        double cc, cs;
        chirp(n, a.Nchirp, cc, cs);
        const double r = c * cc + sn * cs, i = sn * cc - c * cs;
        c = r;
        sn = i;
    }
    const int64_t nn = a.ck_t ? (n % a.L2) * a.L1 + n / a.L2 : n;
    ((cx<T> *)a.ck)[b * a.ck_bs + nn] = cmul_d(x, c, sn);
}

// spectral multiplier of a row pass (see RowArgs)
template <typename T>
__device__ __forceinline__ cx<T> row_mid(cx<T> x, const RowArgs &a, int64_t pos)
{
    if (a.bhat) {
        const double br = a.bhat[2 * pos], bi = a.conj_tab ? -a.bhat[2 * pos + 1] : a.bhat[2 * pos + 1];
        return cmul_d(x, br, bi);
    }
    const int m = a.s[pos];
    return cmul_d(x, a.ktab[2 * m], a.ktab[2 * m + 1]);
}

}  // namespace lt
