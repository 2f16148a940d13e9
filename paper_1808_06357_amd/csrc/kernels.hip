// HIP kernels for Strang splitting on lattices, written for CDNA4 (gfx950).
//
// One Strang step on lattice values (eq. (StrangTDSE), Algorithm 1, applied
// in the point domain) is  u <- P u;  U = F u;  U <- K U;  u = F^-1 U;  u <- P u.
// Nothing on this path is a dense contraction, so no MFMA is used: every
// kernel streams complex data through LDS-resident mixed-radix Stockham
// FFTs (radices 2..16) and is bounded by HBM / Infinity-Cache bandwidth.
//
// Transform layouts (all in place in one buffer of L complex numbers):
//  * one-workgroup ("resident") runs: the whole transform and the whole step
//    loop stay in LDS;
//  * two-pass runs: the buffer is an L1 x L2 row-major matrix.  A column pass
//    transforms C adjacent columns (length L1) per workgroup, a row pass
//    transforms rows (length L2).  For rank-1 lattices this is the four-step
//    FFT (twiddle W_L^{n2 k1} between the passes, spectrum index
//    k1 + L1 k2 stored at k1 L2 + k2); for rank-2 lattices it is the 2-D DFT
//    of eq. (Fnx) and needs no twiddle.
//  * The kinetic phase sits in the row pass (spectral side), the potential
//    phase in the column pass (point side); the inverse transform uses
//    F^-1 x = conj(F conj(x)), so only forward butterflies exist.
//  * Prime N uses Bluestein's chirp-z identity k xi = (k^2 + xi^2 - (xi-k)^2)/2:
//    each DFT becomes a length-L cyclic convolution with a precomputed kernel
//    spectrum; the chirps of consecutive transforms cancel, so inside the step
//    loop only the masked K and P^2 multiplies remain.
#include <hip/hip_runtime.h>

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

// exp(-i a) for a double angle: reduce a mod 2 pi in double (Cody-Waite split
// of 2 pi), then sincos in double.
__device__ __forceinline__ void expm_i(double a, double &c, double &s)
{
    const double inv2pi = 0.15915494309189533577;
    const double twopi_hi = 6.28318530717958623200;    // 2 pi rounded to double
    const double twopi_lo = 2.44929359829470635445e-16; // 2 pi - twopi_hi
    double q = rint(a * inv2pi);
    double r = __fma_rn(-q, twopi_hi, a);
    r = __fma_rn(-q, twopi_lo, r);
    double sn, cs;
    sincos(r, &sn, &cs);
    c = cs;
    s = -sn;
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

template <typename T>
__device__ __forceinline__ cx<T> to_cx(double c, double s) { return {(T)c, (T)s}; }

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

template <typename T>
struct Dft<T, 8> {
    static __device__ __forceinline__ void run(cx<T> *v)
    {
        const T r = (T)0.70710678118654752440084436210484904;
        cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, 4>::run(e);
        Dft<T, 4>::run(o);
        o[1] = {(o[1].x + o[1].y) * r, (o[1].y - o[1].x) * r};
        o[2] = mul_negi(o[2]);
        o[3] = {(o[3].y - o[3].x) * r, -(o[3].x + o[3].y) * r};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = e[k] + o[k];
            v[k + 4] = e[k] - o[k];
        }
    }
};

// cos / sin of 2 pi m / 16 for the radix-16 inner twiddles
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
__device__ __forceinline__ constexpr double s16(int m) { return c16((m + 12) & 15); }  // sin = cos(x - pi/2)

template <typename T>
struct Dft<T, 16> {
    // 16 = 4 x 4: four radix-4 DFTs over j2 (stride 4), twiddle W16^{j1 k2},
    // four radix-4 DFTs over j1.
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
                if (j1 == 0) continue;
                const int m = j1 * k2;
                const cx<T> w = {(T)c16(m), (T)(-s16(m))};
                a[j1][k2] = cmul(a[j1][k2], w);
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
                const T c = (T)cosr<R>(m), s = (T)sinr<R>(m);
                re += a[j - 1].x * c + b[j - 1].y * s;
                im += a[j - 1].y * c - b[j - 1].x * s;
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

// ---------------------------------------------------------------- Stockham stage in LDS
// One radix-R stage over `nseq` sequences of length L stored at
// s[q*ss + e*es]; Ns = product of the radices already applied.  Butterfly t
// reads elements t + r L/R, applies W_{Ns R}^{(t mod Ns) r}, and writes
// positions (t - t mod Ns) R + (t mod Ns) + r Ns (autosorting Stockham; the
// result after the last stage is in natural order).  All reads of a stage
// finish before any write (one barrier between), so the stage is in place.
template <typename T, int R, int EPT>
__device__ __forceinline__ void stage(cx<T> *s, int L, int nseq, int es, int ss, bool seqfast,
                                      int Ns, const cx<T> *__restrict__ tw)
{
    constexpr int J = (EPT + R - 1) / R;
    const int bps = L / R;
    const int nb = nseq * bps;
    const int twstep = L / (Ns * R);
    cx<T> v[J][R];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int b = threadIdx.x + j * kThreads;
        if (b < nb) {
            int q, t;
            if (seqfast) { q = b % nseq; t = b / nseq; }
            else { t = b % bps; q = b / bps; }
            const cx<T> *base = s + q * ss;
            const int jj = t % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[j][r] = base[(t + r * bps) * es];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[j][r] = cmul(v[j][r], tw[jj * r * twstep]);
            }
            Dft<T, R>::run(v[j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int b = threadIdx.x + j * kThreads;
        if (b < nb) {
            int q, t;
            if (seqfast) { q = b % nseq; t = b / nseq; }
            else { t = b % bps; q = b / bps; }
            cx<T> *base = s + q * ss;
            const int jj = t % Ns;
            const int ob = (t - jj) * R + jj;
#pragma unroll
            for (int r = 0; r < R; ++r) base[(ob + r * Ns) * es] = v[j][r];
        }
    }
    __syncthreads();
}

// Forward unnormalised DFT of nseq sequences in LDS (caller has synchronised
// after filling s).  tw[q] = W_L^q.
template <typename T, int EPT>
__device__ void fft_lds(cx<T> *s, const Radices &rd, int nseq, int es, int ss, bool seqfast,
                        const cx<T> *__restrict__ tw)
{
    const int L = rd.L;
    int Ns = 1;
    for (int st = 0; st < rd.n; ++st) {
        const int R = rd.r[st];
        switch (R) {
        case 2: stage<T, 2, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        case 3: stage<T, 3, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        case 4: stage<T, 4, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        case 5: stage<T, 5, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        case 7: stage<T, 7, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        case 8: stage<T, 8, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        case 16: stage<T, 16, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw); break;
        default: break;
        }
        Ns *= R;
    }
}

// four-step twiddle W_L^{n2 k1}, L = L1 L2, from two double tables
template <typename T>
__device__ __forceinline__ cx<T> tw4(int n2, int k1, int L2, const double *hi, const double *lo)
{
    const int64_t q = (int64_t)n2 * k1;
    const int qa = (int)(q / L2), qb = (int)(q - (int64_t)qa * L2);
    const double ax = hi[2 * qa], ay = hi[2 * qa + 1], bx = lo[2 * qb], by = lo[2 * qb + 1];
    return {(T)(ax * bx - ay * by), (T)(ax * by + ay * bx)};
}

template <typename T>
__device__ __forceinline__ cx<T> ldc(const void *p, int64_t i) { return ((const cx<T> *)p)[i]; }

// ---------------------------------------------------------------- column pass
// C adjacent columns of the L1 x L2 buffer per workgroup (tile index x),
// batch item y.  Optional steps, in order:
//   pre_inv : x <- conj(x) W(n2,k1); column DFT; conj        (inverse of the row side)
//   mid     : point-domain work at natural index n = n1 L2 + n2
//   post_fwd: column DFT; x <- x W(n2,k1)                    (forward towards the rows)
// In adjoint mode the tile also holds the cotangent columns (sequences C..2C-1).
template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_col(ColArgs a)
{
    extern __shared__ char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int L1 = a.L1, L2 = a.L2, C = a.C;
    const int nvec = a.adjoint ? 2 : 1;
    const int Cq = C * nvec;                  // sequences in the tile
    const int tile = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int c0 = tile * C;
    const int cw = min(C, L2 - c0);           // valid columns in this tile
    const int tot = L1 * Cq;
    cx<T> *buf0 = (cx<T> *)a.buf + b * a.buf_bs;
    cx<T> *buf1 = a.adjoint ? (cx<T> *)a.buf2 + b * a.buf2_bs : nullptr;
    const cx<T> *twa = (const cx<T> *)a.twa;

    // ---- load
    for (int e = threadIdx.x; e < tot; e += kThreads) {
        const int q = e % Cq, n1 = e / Cq;
        const int vec = q / C, qc = q - vec * C;
        cx<T> x = {0, 0};
        if (qc < cw) {
            const int n2 = c0 + qc;
            const int64_t gi = (int64_t)n1 * L2 + n2;
            if (a.pre_inv) {
                x = vec ? buf1[gi] : buf0[gi];
                x = conjg(x);
                if (a.twiddle) x = cmul(x, tw4<T>(n2, n1, L2, a.tw4hi, a.tw4lo));
            } else {
                const void *src = vec ? a.in2 : a.in;
                const int64_t bs = vec ? a.in2_bs : a.in_bs;
                if (src) x = gi < a.Nvalid ? ldc<T>(src, b * bs + gi) : cx<T>{0, 0};
                else x = vec ? buf1[gi] : buf0[gi];
            }
        }
        s[e] = x;
    }
    __syncthreads();
    if (a.pre_inv) fft_lds<T, EPT>(s, a.rad, Cq, Cq, 1, true, twa);

    // ---- point-domain work (natural index n)
    const double *vb = a.v ? a.v + b * a.v_bs : nullptr;
    for (int e = threadIdx.x; e < L1 * C; e += kThreads) {
        const int qc = e % C, n1 = e / C;
        if (qc >= cw) continue;
        const int64_t n = (int64_t)n1 * L2 + c0 + qc;
        const int e0 = n1 * Cq + qc;
        cx<T> x = s[e0];
        if (a.pre_inv) x = conjg(x);
        if (n >= a.Nvalid) {
            s[e0] = {0, 0};
            if (a.adjoint) s[e0 + C] = {0, 0};
            continue;
        }
        if (!a.adjoint) {
            if (a.ck) {  // lattice value u = x exp(-i ck_phase v) [conj(c_n)]
                double c, sn;
                expm_i(a.ck_phase * a.ck_v[b * a.v_bs + n], c, sn);
                cx<T> w = to_cx<T>(c, sn);
                if (a.ck_chirp) {
                    double cc, cs;
                    chirp(n, a.Nchirp, cc, cs);
                    w = cmul(w, to_cx<T>(cc, -cs));
                }
                ((cx<T> *)a.ck)[b * a.ck_bs + n] = cmul(x, w);
            }
            if (a.tab) x = cmul(x, ldc<T>(a.tab, b * a.tab_bs + n));
            if (vb) {
                double c, sn;
                expm_i(a.phase * vb[n], c, sn);
                cx<T> w = to_cx<T>(c, sn);
                if (a.chirp) {
                    double cc, cs;
                    chirp(n, a.Nchirp, cc, cs);
                    w = cmul(w, to_cx<T>(cc, a.chirp > 0 ? cs : -cs));
                }
                x = cmul(x, w);
            }
            if (a.scale != 1.0) x = scal(x, (T)a.scale);
            if (a.out) ((cx<T> *)a.out)[b * a.out_bs + n] = x;
            else s[e0] = x;
        } else {
            // adjoint: x = state-side value (a, up to a unit chirp), y = cotangent side (mu)
            cx<T> y = s[e0 + C];
            if (a.pre_inv) y = conjg(y);
            double c, sn;
            expm_i(a.phase * vb[n], c, sn);          // backward phase exp(-i phase v)
            cx<T> w = to_cx<T>(c, sn);
            if (a.reset) {
                // state from the checkpoint: a = conj(w_half) ckpt, in transform units
                double rc, rs;
                expm_i(a.reset_phase * vb[n], rc, rs);
                cx<T> rw = to_cx<T>(rc, rs);
                if (a.chirp) {
                    double cc, cs;
                    chirp(n, a.Nchirp, cc, cs);
                    rw = cmul(rw, to_cx<T>(cc, cs));
                }
                x = cmul(ldc<T>(a.reset, b * a.reset_bs + n), rw);
            }
            // Im(conj(mu) a) is chirp invariant (|c_n| = 1)
            const double im = (double)y.x * (double)x.y - (double)y.y * (double)x.x;
            a.gacc[b * a.gacc_bs + n] += a.gcoef * im;
            if (a.adjoint == 3) {
                // last: dJ/du0 = w * conj(c_n) * y
                if (a.chirp) {
                    double cc, cs;
                    chirp(n, a.Nchirp, cc, cs);
                    w = cmul(w, to_cx<T>(cc, -cs));
                }
                ((cx<T> *)a.out2)[b * a.out2_bs + n] = cmul(y, w);
                continue;
            }
            if (a.adjoint == 1 && a.chirp) {
                double cc, cs;
                chirp(n, a.Nchirp, cc, cs);
                w = cmul(w, to_cx<T>(cc, cs));
            }
            if (a.adjoint == 2 && a.tab) w = ldc<T>(a.tab, b * a.tab_bs + n);
            if (a.scale != 1.0) w = scal(w, (T)a.scale);
            s[e0] = cmul(x, w);
            s[e0 + C] = cmul(y, w);
        }
    }
    if (!a.post_fwd) return;
    __syncthreads();
    fft_lds<T, EPT>(s, a.rad, Cq, Cq, 1, true, twa);

    // ---- store
    for (int e = threadIdx.x; e < tot; e += kThreads) {
        const int q = e % Cq, k1 = e / Cq;
        const int vec = q / C, qc = q - vec * C;
        if (qc >= cw) continue;
        const int n2 = c0 + qc;
        const int64_t gi = (int64_t)k1 * L2 + n2;
        cx<T> x = s[e];
        if (a.twiddle) x = cmul(x, tw4<T>(n2, k1, L2, a.tw4hi, a.tw4lo));
        if (vec) buf1[gi] = x;
        else buf0[gi] = x;
    }
}

// ---------------------------------------------------------------- row pass
// `rows` contiguous rows of length L2 per workgroup: DFT; x <- x * tab
// (tab or conj(tab), spectral position k1 L2 + k2); inverse DFT.
template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_row(RowArgs a)
{
    extern __shared__ char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int L2 = a.L2;
    const int r0 = blockIdx.x * a.rows;
    const int rw = min(a.rows, a.L1 - r0);
    const int64_t b = blockIdx.y;
    cx<T> *buf = (cx<T> *)a.buf + b * a.buf_bs + (int64_t)r0 * L2;
    const cx<T> *twb = (const cx<T> *)a.twb;
    const int tot = a.rows * L2;
    for (int e = threadIdx.x; e < tot; e += kThreads)
        s[e] = (e / L2) < rw ? buf[e] : cx<T>{0, 0};
    __syncthreads();
    fft_lds<T, EPT>(s, a.rad, a.rows, 1, L2, false, twb);
    if (a.fft_only) {
        for (int e = threadIdx.x; e < rw * L2; e += kThreads) buf[e] = s[e];
        return;
    }
    const cx<T> *tab = (const cx<T> *)a.tab + b * a.tab_bs + (int64_t)r0 * L2;
    for (int e = threadIdx.x; e < rw * L2; e += kThreads) {
        cx<T> t = tab[e];
        if (a.conj_tab) t = conjg(t);
        s[e] = conjg(cmul(s[e], t));
    }
    __syncthreads();
    fft_lds<T, EPT>(s, a.rad, a.rows, 1, L2, false, twb);
    for (int e = threadIdx.x; e < rw * L2; e += kThreads) buf[e] = conjg(s[e]);
}

// ---------------------------------------------------------------- resident run
// Whole run of one state in one workgroup: the transform (1-D of length L,
// or 2-D n1 x n2) and every step stay in LDS.
template <typename T, int EPT>
__device__ __forceinline__ void res_fft(cx<T> *s, const ResArgs &a)
{
    if (!a.rank2) {
        fft_lds<T, EPT>(s, a.ra, 1, 1, a.L, false, (const cx<T> *)a.twa);
    } else {
        fft_lds<T, EPT>(s, a.rb, a.n1, 1, a.n2, false, (const cx<T> *)a.twb);  // rows
        fft_lds<T, EPT>(s, a.ra, a.n2, a.n2, 1, true, (const cx<T> *)a.twa);  // columns
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_resident(ResArgs a)
{
    extern __shared__ char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int64_t b = blockIdx.x;
    const int L = (int)a.L;
    const int N = (int)a.N;
    cx<T> *u = (cx<T> *)a.u + b * a.u_bs;
    const double *vb = a.v + b * a.v_bs;
    const cx<T> *P2 = a.tabP2 ? (const cx<T> *)a.tabP2 + b * a.p2_bs : nullptr;
    const cx<T> *K = (const cx<T> *)a.tabK;
    const cx<T> *B = (const cx<T> *)a.bhat;

    // first half potential step (times the chirp for chirp-z)
    for (int n = threadIdx.x; n < L; n += kThreads) {
        cx<T> x = {0, 0};
        if (n < N) {
            x = u[n];
            if (a.ck) ((cx<T> *)a.ck)[b * N + n] = x;
            double c, sn;
            expm_i(a.phase_half * vb[n], c, sn);
            cx<T> w = to_cx<T>(c, sn);
            if (a.bluestein) {
                double cc, cs;
                chirp(n, N, cc, cs);
                w = cmul(w, to_cx<T>(cc, cs));
            }
            x = cmul(x, w);
        }
        s[n] = x;
    }
    __syncthreads();
    for (int64_t st = 0; st < a.steps; ++st) {
        res_fft<T, EPT>(s, a);
        const cx<T> *M1 = a.bluestein ? B : K;
        for (int n = threadIdx.x; n < L; n += kThreads) s[n] = conjg(cmul(s[n], M1[n]));
        __syncthreads();
        res_fft<T, EPT>(s, a);
        if (a.bluestein) {
            for (int n = threadIdx.x; n < L; n += kThreads)
                s[n] = n < N ? cmul(conjg(s[n]), K[n]) : cx<T>{0, 0};
            __syncthreads();
            res_fft<T, EPT>(s, a);
            for (int n = threadIdx.x; n < L; n += kThreads) s[n] = conjg(cmul(s[n], conjg(B[n])));
            __syncthreads();
            res_fft<T, EPT>(s, a);
        }
        const bool last = st == a.steps - 1;
        const bool ckpt = a.ck && !last && ((st + 1) % a.ck_every == 0);
        for (int n = threadIdx.x; n < L; n += kThreads) {
            cx<T> x = conjg(s[n]);
            if (n >= N) { s[n] = {0, 0}; continue; }
            if (last || ckpt) {
                double c, sn;
                expm_i(a.phase_half * vb[n], c, sn);
                cx<T> w = to_cx<T>(c, sn);
                if (a.bluestein) {
                    double cc, cs;
                    chirp(n, N, cc, cs);
                    w = cmul(w, to_cx<T>(cc, -cs));
                }
                const cx<T> un = cmul(x, w);
                if (last) { u[n] = un; continue; }
                ((cx<T> *)a.ck)[((st + 1) / a.ck_every) * a.ck_stride + b * N + n] = un;
            }
            s[n] = cmul(x, P2[n]);
        }
        __syncthreads();
    }
}

// single forward DFT of one sequence (plan-time helper)
template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_fft_single(Radices ra, const void *twa, void *buf)
{
    extern __shared__ char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *g = (cx<T> *)buf;
    for (int n = threadIdx.x; n < ra.L; n += kThreads) s[n] = g[n];
    __syncthreads();
    fft_lds<T, EPT>(s, ra, 1, 1, ra.L, false, (const cx<T> *)twa);
    for (int n = threadIdx.x; n < ra.L; n += kThreads) g[n] = s[n];
}

// ---------------------------------------------------------------- tables
// kinetic multipliers exp(-i kin * s_chi) * scale at the row-pass position
// (transposed: position k1 L2 + k2 holds chi = k1 + L1 k2)
template <typename T>
__global__ void k_kinetic_table(cx<T> *dst, const int32_t *s_key, int64_t N, int L1, int L2,
                                int transposed, double kin, double scale)
{
    for (int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pos < N;
         pos += (int64_t)gridDim.x * blockDim.x) {
        int64_t chi = pos;
        if (transposed) {
            const int64_t k1 = pos / L2, k2 = pos - k1 * L2;
            chi = k1 + (int64_t)L1 * k2;
        }
        double c, sn;
        expm_i(kin * (double)s_key[chi], c, sn);
        dst[pos] = to_cx<T>(c * scale, sn * scale);
    }
}

template <typename T>
__global__ void k_phase_table(cx<T> *dst, const double *v, int64_t v_bs, int64_t N, int batch,
                              double phase)
{
    const int64_t total = N * batch;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / N, n = i - b * N;
        double c, sn;
        expm_i(phase * v[b * v_bs + n], c, sn);
        dst[i] = to_cx<T>(c, sn);
    }
}

// natural-order double spectrum -> schedule layout in the run precision
template <typename T>
__global__ void k_convert_permute(cx<T> *dst, const cx<double> *src, int64_t L, int L1, int L2,
                                  int transposed, double scale)
{
    for (int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pos < L;
         pos += (int64_t)gridDim.x * blockDim.x) {
        int64_t xi = pos;
        if (transposed) {
            const int64_t k1 = pos / L2, k2 = pos - k1 * L2;
            xi = k1 + (int64_t)L1 * k2;
        }
        const cx<double> z = src[xi];
        dst[pos] = {(T)(z.x * scale), (T)(z.y * scale)};
    }
}

__global__ void k_unpermute(cx<double> *dst, const cx<double> *src, int64_t L, int L1, int L2)
{
    for (int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pos < L;
         pos += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k1 = pos / L2, k2 = pos - k1 * L2;
        dst[k1 + (int64_t)L1 * k2] = src[pos];
    }
}

// chirp-z kernel b_j = conj(c_j) for |j| < N, wrapped cyclically into length L
__global__ void k_chirp_filter(cx<double> *dst, int64_t N, int64_t L)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < L;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = -1;
        if (j < N) m = j;
        else if (j > L - N) m = L - j;
        cx<double> z = {0.0, 0.0};
        if (m >= 0) {
            double c, s;
            chirp(m, N, c, s);
            z = {c, -s};
        }
        dst[j] = z;
    }
}

__global__ void k_reduce_batch(double *dst, const double *src, int64_t N, int batch)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int b = 0; b < batch; ++b) acc += src[(int64_t)b * N + n];
        dst[n] = acc;
    }
}

// ---------------------------------------------------------------- launchers
static inline size_t esize(int prec) { return prec == LT_C128 ? 16 : 8; }

static int grid1d(int64_t n)
{
    int64_t g = (n + 255) / 256;
    return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

int kernels_init()
{
    static int done = 0;
    if (done) return 0;
    done = 1;
    const int lim = 160 * 1024;
    hipFuncSetAttribute((const void *)k_col<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_col<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_resident<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_resident<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipGetLastError();
    return 0;
}

int launch_col(int prec, const Sched &s, const ColArgs &a, int batch, void *stream)
{
    const int nvec = a.adjoint ? 2 : 1;
    const size_t lds = (size_t)a.L1 * a.C * nvec * esize(prec);
    dim3 grid(a.ntiles, batch);
    if (prec == LT_C128)
        hipLaunchKernelGGL((k_col<double, 16>), grid, dim3(kThreads), lds, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((k_col<float, 32>), grid, dim3(kThreads), lds, (hipStream_t)stream, a);
    (void)s;
    return (int)hipGetLastError();
}

int launch_row(int prec, const Sched &s, const RowArgs &a, int batch, void *stream)
{
    const size_t lds = (size_t)a.rows * a.L2 * esize(prec);
    dim3 grid(a.nblk, batch);
    if (prec == LT_C128)
        hipLaunchKernelGGL((k_row<double, 16>), grid, dim3(kThreads), lds, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((k_row<float, 32>), grid, dim3(kThreads), lds, (hipStream_t)stream, a);
    (void)s;
    return (int)hipGetLastError();
}

int launch_resident(int prec, const Sched &s, const ResArgs &a, int batch, void *stream)
{
    const size_t lds = (size_t)a.L * esize(prec);
    if (prec == LT_C128)
        hipLaunchKernelGGL((k_resident<double, 16>), dim3(batch), dim3(kThreads), lds,
                           (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL((k_resident<float, 32>), dim3(batch), dim3(kThreads), lds,
                           (hipStream_t)stream, a);
    (void)s;
    return (int)hipGetLastError();
}

int launch_fft_single(int prec, const Radices &ra, const void *twa, void *buf, int64_t L, void *stream)
{
    const size_t lds = (size_t)L * esize(prec);
    if (prec == LT_C128)
        hipLaunchKernelGGL((k_fft_single<double, 16>), dim3(1), dim3(kThreads), lds,
                           (hipStream_t)stream, ra, twa, buf);
    else
        hipLaunchKernelGGL((k_fft_single<float, 32>), dim3(1), dim3(kThreads), lds,
                           (hipStream_t)stream, ra, twa, buf);
    return (int)hipGetLastError();
}

int launch_setup_kernel_table(int prec, void *dst, const int32_t *s_key, int64_t N, int L1, int L2,
                              int transposed, double kin, double scale, void *stream)
{
    if (prec == LT_C128)
        hipLaunchKernelGGL(k_kinetic_table<double>, dim3(grid1d(N)), dim3(256), 0, (hipStream_t)stream,
                           (cx<double> *)dst, s_key, N, L1, L2, transposed, kin, scale);
    else
        hipLaunchKernelGGL(k_kinetic_table<float>, dim3(grid1d(N)), dim3(256), 0, (hipStream_t)stream,
                           (cx<float> *)dst, s_key, N, L1, L2, transposed, kin, scale);
    return (int)hipGetLastError();
}

int launch_setup_phase_table(int prec, void *dst, const double *v, int64_t v_bs, int64_t N, int batch,
                             double phase, void *stream)
{
    if (prec == LT_C128)
        hipLaunchKernelGGL(k_phase_table<double>, dim3(grid1d(N * batch)), dim3(256), 0,
                           (hipStream_t)stream, (cx<double> *)dst, v, v_bs, N, batch, phase);
    else
        hipLaunchKernelGGL(k_phase_table<float>, dim3(grid1d(N * batch)), dim3(256), 0,
                           (hipStream_t)stream, (cx<float> *)dst, v, v_bs, N, batch, phase);
    return (int)hipGetLastError();
}

int launch_convert_permute(int prec_dst, void *dst, const void *src, int64_t L, int L1, int L2,
                           int transposed, double scale, void *stream)
{
    if (prec_dst == LT_C128)
        hipLaunchKernelGGL(k_convert_permute<double>, dim3(grid1d(L)), dim3(256), 0, (hipStream_t)stream,
                           (cx<double> *)dst, (const cx<double> *)src, L, L1, L2, transposed, scale);
    else
        hipLaunchKernelGGL(k_convert_permute<float>, dim3(grid1d(L)), dim3(256), 0, (hipStream_t)stream,
                           (cx<float> *)dst, (const cx<double> *)src, L, L1, L2, transposed, scale);
    return (int)hipGetLastError();
}

int launch_unpermute_c128(void *dst_nat, const void *src, int64_t L, int L1, int L2, void *stream)
{
    hipLaunchKernelGGL(k_unpermute, dim3(grid1d(L)), dim3(256), 0, (hipStream_t)stream,
                       (cx<double> *)dst_nat, (const cx<double> *)src, L, L1, L2);
    return (int)hipGetLastError();
}

int launch_chirp_filter(void *dst, int64_t N, int64_t L, void *stream)
{
    hipLaunchKernelGGL(k_chirp_filter, dim3(grid1d(L)), dim3(256), 0, (hipStream_t)stream,
                       (cx<double> *)dst, N, L);
    return (int)hipGetLastError();
}

int launch_reduce_batch(double *dst, const double *src, int64_t N, int batch, void *stream)
{
    hipLaunchKernelGGL(k_reduce_batch, dim3(grid1d(N)), dim3(256), 0, (hipStream_t)stream, dst, src,
                       N, batch);
    return (int)hipGetLastError();
}

}  // namespace lt
