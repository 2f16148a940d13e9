// HIP kernels for Strang splitting on lattices, written for CDNA4 (gfx950):
// the general (any 7-smooth length) LDS Stockham kernels, the plan-time
// table kernels and all launchers.
//
// One Strang step on lattice values (eq. (StrangTDSE), Algorithm 1, applied
// in the point domain) is  u <- P u;  U = F u;  U <- K U;  u = F^-1 U;  u <- P u.
// Nothing on this path is a dense contraction, so no MFMA is used: every
// kernel streams complex data through LDS-resident mixed-radix Stockham
// FFTs (radices 2..16) and is bounded by memory bandwidth.
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
//    phase in the column pass (point side), both evaluated in FP64 on the
//    fly; the inverse transform uses F^-1 x = conj(F conj(x)), so only forward
//    butterflies exist.
//  * Prime N uses Bluestein's chirp-z identity k xi = (k^2 + xi^2 - (xi-k)^2)/2:
//    each DFT becomes a length-L cyclic convolution with a precomputed kernel
//    spectrum; the chirps of consecutive transforms cancel, so inside the step
//    loop only the masked K and P^2 multiplies remain.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "device.h"
#include "lt_internal.h"

namespace lt {

// ---------------------------------------------------------------- Stockham stage in LDS
// One radix-R stage over `nseq` sequences of length L stored at
// s[q*ss + e*es]; Ns = product of the radices already applied.  Butterfly t
// reads elements t + r L/R, applies W_{Ns R}^{(t mod Ns) r}, and writes
// positions (t - t mod Ns) R + (t mod Ns) + r Ns (autosorting Stockham; the
// result after the last stage is in natural order).  All reads of a stage
// finish before any write (one barrier between), so the stage is in place.
// Kept out of line: each radix's butterflies then get registers of their own
// instead of one allocation covering every radix of the dispatch below.
template <typename T, int R, int EPT>
__device__ __attribute__((noinline)) void stage(cx<T> *s, int L, int nseq, int es, int ss, bool seqfast,
                                                int Ns, const Tw<T> *__restrict__ tw)
{
    constexpr int J = (EPT + R - 1) / R;
    const int bps = L / R;
    const int nb = nseq * bps;
    const int twstep = L / (Ns * R);
    const int in_stride = bps * es, out_stride = Ns * es;
    const FDiv dq = fdiv_make(seqfast ? nseq : bps), dns = fdiv_make(Ns);
    cx<T> v[J][R];
    int obase[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int b = threadIdx.x + j * kThreads;
        obase[j] = -1;
        if (b < nb) {
            int q, t;
            if (seqfast) { t = fdiv(b, dq); q = b - t * nseq; }
            else { q = fdiv(b, dq); t = b - q * bps; }
            const int jj = t - fdiv(t, dns) * Ns;
            const int ib = q * ss + t * es;
            obase[j] = q * ss + ((t - jj) * R + jj) * es;
#pragma unroll
            for (int r = 0; r < R; ++r) v[j][r] = s[ib + r * in_stride];
            if (Ns > 1) {
                // W_{Ns R}^{jj r}: one table entry per butterfly, its powers in double
                const cx<double> w = tw_d(tw[jj * twstep]);
                double pr[R], pi[R];
                powers<R>(w.x, w.y, pr, pi);
#pragma unroll
                for (int r = 1; r < R; ++r) v[j][r] = cmul_d(v[j][r], pr[r], pi[r]);
            }
            Dft<T, R>::run(v[j]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (obase[j] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) s[obase[j] + r * out_stride] = v[j][r];
        }
    }
    __syncthreads();
}

// Forward unnormalised DFT of nseq sequences in LDS (caller has synchronised
// after filling s).  tw[q] = W_L^q.
template <typename T, int EPT>
__device__ void fft_lds(cx<T> *s, const Radices &rd, int nseq, int es, int ss, bool seqfast,
                        const Tw<T> *__restrict__ tw)
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
        case 16:  // float only: the double schedules stop at radix 8
            if constexpr (sizeof(T) == 4) stage<T, 16, EPT>(s, L, nseq, es, ss, seqfast, Ns, tw);
            break;
        default: break;
        }
        Ns *= R;
    }
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
__device__ void col_body(const ColArgs &a, int tile, int64_t b, cx<T> *s)
{
    const int L1 = a.L1, L2 = a.L2, C = a.C;
    const int nvec = a.adjoint ? 2 : 1;
    const int Cq = C * nvec;                  // sequences in the tile
    const int c0 = tile * C;
    const int cw = min(C, L2 - c0);           // valid columns in this tile
    const int tot = L1 * Cq;
    const FDiv dCq = fdiv_make(Cq), dC = fdiv_make(C), dL2 = fdiv_make(L2);
    cx<T> *buf0 = (cx<T> *)a.buf + b * a.buf_bs;
    cx<T> *buf1 = a.adjoint ? (cx<T> *)a.buf2 + b * a.buf2_bs : nullptr;
    const Tw<T> *twa = (const Tw<T> *)a.twa;

    // ---- load
    for (int e = threadIdx.x; e < tot; e += kThreads) {
        const int n1 = fdiv(e, dCq), q = e - n1 * Cq;
        const int vec = q >= C, qc = q - vec * C;
        cx<T> x = {0, 0};
        if (qc < cw) {
            const int n2 = c0 + qc;
            const int64_t gi = (int64_t)n1 * L2 + n2;
            if (a.pre_inv) {
                x = vec ? buf1[gi] : buf0[gi];
                x = conjg(x);
                if (a.twiddle) x = tw4mul(x, n2, n1, dL2, a.tw4hi, a.tw4lo);
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
    const double *vb2 = a.v && a.v2 ? a.v2 + b * a.v_bs : nullptr;
    const double *sv = a.sum_part ? a.sum_v + b * a.v_bs : nullptr;
    double s1 = 0.0, s2 = 0.0;
    for (int e = threadIdx.x; e < L1 * C; e += kThreads) {
        const int n1 = fdiv(e, dC), qc = e - n1 * C;
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
            if (a.ck) col_checkpoint(x, a, b, n);
            if (sv) {
                const double q = (double)x.x * (double)x.x + (double)x.y * (double)x.y;
                s1 += q;
                s2 += sv[n] * q;
            }
            x = col_mid(x, a, vb, vb2, n);
            if (a.out) ((cx<T> *)a.out)[b * a.out_bs + n] = x;
            else s[e0] = x;
        } else {
            // adjoint: x = state-side value (a, up to a unit chirp), y = cotangent side (mu)
            cx<T> y = s[e0 + C];
            if (a.pre_inv) y = conjg(y);
            if (a.reset) {
                // state from the checkpoint: a = exp(-i reset_phase v) ckpt (times c_n for chirp-z)
                double rc, rs;
                expm_i(a.reset_phase * vb[n], rc, rs);
                if (a.chirp) {
                    double cc, cs;
                    chirp(n, a.Nchirp, cc, cs);
                    const double r = rc * cc - rs * cs, i = rc * cs + rs * cc;
                    rc = r;
                    rs = i;
                }
                const int64_t rn = a.reset_t ? (int64_t)(c0 + qc) * L1 + n1 : n;
                x = cmul_d(ldc<T>(a.reset, b * a.reset_bs + rn), rc, rs);
            }
            // Im(conj(mu) a) is chirp invariant (|c_n| = 1)
            const double im = (double)y.x * (double)x.y - (double)y.y * (double)x.x;
            a.gacc[b * a.gacc_bs + n] += a.gcoef * im;
            double c, sn;
            expm_i(a.phase * vb[n], c, sn);            // backward phase exp(-i phase v)
            if (a.adjoint == 3) {
                // last: dJ/du0 = exp(-i phase v) conj(c_n) mu
                if (a.chirp) {
                    double cc, cs;
                    chirp(n, a.Nchirp, cc, cs);
                    const double r = c * cc + sn * cs, i = sn * cc - c * cs;
                    c = r;
                    sn = i;
                }
                ((cx<T> *)a.out2)[b * a.out2_bs + n] = cmul_d(y, c, sn);
                continue;
            }
            if (a.adjoint == 1 && a.chirp) {
                double cc, cs;
                chirp(n, a.Nchirp, cc, cs);
                const double r = c * cc - sn * cs, i = c * cs + sn * cc;
                c = r;
                sn = i;
            }
            s[e0] = cmul_d(x, c, sn);
            s[e0 + C] = cmul_d(y, c, sn);
        }
    }
    if (a.sum_part) {
        block_sum2<kThreads>(s1, s2);
        if (threadIdx.x == 0) {
            double *pb = a.sum_part + ((int64_t)b * a.sum_pt + tile) * 2;
            pb[0] = s1;
            pb[1] = s2;
        }
    }
    if (!a.post_fwd) return;
    __syncthreads();
    fft_lds<T, EPT>(s, a.rad, Cq, Cq, 1, true, twa);

    // ---- store
    for (int e = threadIdx.x; e < tot; e += kThreads) {
        const int k1 = fdiv(e, dCq), q = e - k1 * Cq;
        const int vec = q >= C, qc = q - vec * C;
        if (qc >= cw) continue;
        const int n2 = c0 + qc;
        const int64_t gi = (int64_t)k1 * L2 + n2;
        cx<T> x = s[e];
        if (a.twiddle) x = tw4mul(x, n2, k1, dL2, a.tw4hi, a.tw4lo);
        if (vec) buf1[gi] = x;
        else buf0[gi] = x;
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_col(ColArgs a)
{
    extern __shared__ char smem_raw[];
    col_body<T, EPT>(a, blockIdx.x, blockIdx.y, reinterpret_cast<cx<T> *>(smem_raw));
}

// ---------------------------------------------------------------- row pass
// `rows` contiguous rows of length L2 per workgroup: DFT; spectral multiplier;
// inverse DFT.
template <typename T, int EPT>
__device__ void row_body(const RowArgs &a, int blk, int64_t b, cx<T> *s)
{
    const int L2 = a.L2;
    const int r0 = blk * a.rows;
    const int rw = min(a.rows, a.L1 - r0);
    cx<T> *buf = (cx<T> *)a.buf + b * a.buf_bs + (int64_t)r0 * L2;
    const Tw<T> *twb = (const Tw<T> *)a.twb;
    const int tot = a.rows * L2;
    const int valid = rw * L2;
    for (int e = threadIdx.x; e < tot; e += kThreads)
        s[e] = e < valid ? buf[e] : cx<T>{0, 0};
    __syncthreads();
    fft_lds<T, EPT>(s, a.rad, a.rows, 1, L2, false, twb);
    if (a.fft_only) {
        for (int e = threadIdx.x; e < rw * L2; e += kThreads) buf[e] = s[e];
        return;
    }
    const int64_t p0 = (int64_t)r0 * L2;
    for (int e = threadIdx.x; e < rw * L2; e += kThreads) s[e] = conjg(row_mid(s[e], a, p0 + e));
    __syncthreads();
    fft_lds<T, EPT>(s, a.rad, a.rows, 1, L2, false, twb);
    for (int e = threadIdx.x; e < rw * L2; e += kThreads) buf[e] = conjg(s[e]);
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_row(RowArgs a)
{
    extern __shared__ char smem_raw[];
    row_body<T, EPT>(a, blockIdx.x, blockIdx.y, reinterpret_cast<cx<T> *>(smem_raw));
}

// ---------------------------------------------------------------- resident run
// Whole run of one state in one workgroup: the transform (1-D of length L,
// or 2-D n1 x n2) and every step stay in LDS.
template <typename T, int EPT>
__device__ __forceinline__ void res_fft(cx<T> *s, const ResArgs &a)
{
    if (!a.rank2) {
        fft_lds<T, EPT>(s, a.ra, 1, 1, a.L, false, (const Tw<T> *)a.twa);
    } else {
        fft_lds<T, EPT>(s, a.rb, a.n1, 1, a.n2, false, (const Tw<T> *)a.twb);  // rows
        fft_lds<T, EPT>(s, a.ra, a.n2, a.n2, 1, true, (const Tw<T> *)a.twa);  // columns
    }
}

template <typename T, int EPT>
__device__ void resident_body(const ResArgs &a, int64_t b, cx<T> *s)
{
    const int L = (int)a.L;
    const int N = (int)a.N;
    cx<T> *u = (cx<T> *)a.u + b * a.u_bs;
    if (a.steps <= 0) return;
    const double *vb = a.v + b * a.v_bs;
    const double *B = a.bhat;

    // per-step sums of |u_j|^2 and v |u_j|^2 (optional)
    double s1 = 0.0, s2 = 0.0;
    auto put_sums = [&](int64_t j) {
        block_sum2<kThreads>(s1, s2);
        if (threadIdx.x == 0) {
            double *pb = a.sum_part + (j * a.batch + b) * 2;
            pb[0] = s1;
            pb[1] = s2;
        }
        s1 = 0.0;
        s2 = 0.0;
    };
    // first half potential step (times the chirp for chirp-z)
    for (int n = threadIdx.x; n < L; n += kThreads) {
        cx<T> x = {0, 0};
        if (n < N) {
            x = u[n];
            if (a.sum_part) {
                const double q = (double)x.x * (double)x.x + (double)x.y * (double)x.y;
                s1 += q;
                s2 += vb[n] * q;
            }
            if (a.ck) ((cx<T> *)a.ck)[b * N + n] = x;
            double c, sn;
            expm_i(a.phase_half * vb[n], c, sn);
            if (a.bluestein) {
                double cc, cs;
                chirp(n, N, cc, cs);
                const double r = c * cc - sn * cs, i = c * cs + sn * cc;
                c = r;
                sn = i;
            }
            x = cmul_d(x, c, sn);
        }
        s[n] = x;
    }
    if (a.sum_part) put_sums(0);
    __syncthreads();
    for (int64_t st = 0; st < a.steps; ++st) {
        res_fft<T, EPT>(s, a);
        if (a.bluestein) {
            for (int n = threadIdx.x; n < L; n += kThreads) s[n] = conjg(cmul_d(s[n], B[2 * n], B[2 * n + 1]));
        } else {
            for (int n = threadIdx.x; n < L; n += kThreads) {
                const int m = a.s[n];
                s[n] = conjg(cmul_d(s[n], a.ktab[2 * m], a.ktab[2 * m + 1]));
            }
        }
        __syncthreads();
        res_fft<T, EPT>(s, a);
        if (a.bluestein) {
            for (int n = threadIdx.x; n < L; n += kThreads) {
                cx<T> x = {0, 0};
                if (n < N) {
                    const int m = a.s[n];
                    x = cmul_d(conjg(s[n]), a.ktab[2 * m], a.ktab[2 * m + 1]);
                }
                s[n] = x;
            }
            __syncthreads();
            res_fft<T, EPT>(s, a);
            for (int n = threadIdx.x; n < L; n += kThreads) s[n] = conjg(cmul_d(s[n], B[2 * n], -B[2 * n + 1]));
            __syncthreads();
            res_fft<T, EPT>(s, a);
        }
        const bool last = st == a.steps - 1;
        const bool ckpt = a.ck && !last && ((st + 1) % a.ck_every == 0);
        for (int n = threadIdx.x; n < L; n += kThreads) {
            cx<T> x = conjg(s[n]);
            if (n >= N) { s[n] = {0, 0}; continue; }
            if (a.sum_part) {
                const double q = (double)x.x * (double)x.x + (double)x.y * (double)x.y;
                s1 += q;
                s2 += vb[n] * q;
            }
            if (last || ckpt) {
                double c, sn;
                expm_i(a.phase_half * vb[n], c, sn);
                if (a.bluestein) {
                    double cc, cs;
                    chirp(n, N, cc, cs);
                    const double r = c * cc + sn * cs, i = sn * cc - c * cs;
                    c = r;
                    sn = i;
                }
                const cx<T> un = cmul_d(x, c, sn);
                if (last) { u[n] = un; continue; }
                ((cx<T> *)a.ck)[((st + 1) / a.ck_every) * a.ck_stride + b * N + n] = un;
            }
            s[n] = mul_expm_i(x, 2.0 * a.phase_half * vb[n]);
        }
        if (a.sum_part) put_sums(st + 1);
        __syncthreads();
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_resident(ResArgs a)
{
    extern __shared__ char smem_raw[];
    resident_body<T, EPT>(a, blockIdx.x, reinterpret_cast<cx<T> *>(smem_raw));
}

// ---------------------------------------------------------------- batches of unrelated problems
// One launch runs pass g of the batch members listed in idx; member k owns
// the blocks [start[k], start[k+1]) of the launch's block range, which begins
// at block `off` (column tiles or row blocks).  A member's role at pass g
// follows its schedule:
//   two passes per step:  g = 0 first, odd g row, other g potential P^2, last g last;
//   chirp-z DFT pairs:    g = 0 first, g = 1, 3 mod 4 row (spectrum, conjugate
//                         spectrum), g = 2 mod 4 kinetic, g = 0 mod 4 potential, last g last.
template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_col_multi(const BatchDesc *d, const int *idx, const int *start,
                                                        int nmem, int nblocks, int off, int64_t g)
{
    extern __shared__ char smem_raw[];
    // the grid is padded to a multiple of 8 blocks (XCD-contiguous tiles)
    const int w = xcd_block(blockIdx.x, gridDim.x);
    if (w >= nblocks) return;
    const int bid = w + off;
    const int k = find_member(start, nmem, bid);
    const BatchDesc &p = d[idx[k]];
    if (g >= p.npass || (g & 1)) return;
    int role;
    if (g == 0) role = 0;
    else if (g == p.npass - 1) role = 3;
    else if (p.bluestein && (g % 4) == 2) role = 2;
    else role = 1;
    col_body<T, EPT>(p.col[role], bid - start[k], 0, reinterpret_cast<cx<T> *>(smem_raw));
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_row_multi(const BatchDesc *d, const int *idx, const int *start,
                                                        int nmem, int off, int64_t g)
{
    extern __shared__ char smem_raw[];
    const int bid = blockIdx.x + off;
    const int k = find_member(start, nmem, bid);
    const BatchDesc &p = d[idx[k]];
    if (g >= p.npass || !(g & 1)) return;
    const int role = (p.bluestein && (g % 4) == 3) ? 1 : 0;
    row_body<T, EPT>(p.row[role], bid - start[k], 0, reinterpret_cast<cx<T> *>(smem_raw));
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kThreads) k_resident_multi(const ResArgs *d)
{
    extern __shared__ char smem_raw[];
    resident_body<T, EPT>(d[blockIdx.x], 0, reinterpret_cast<cx<T> *>(smem_raw));
}

// single forward DFT of one sequence in complex double (plan-time helper)
__global__ void __launch_bounds__(kThreads) k_fft_single(Radices ra, const void *twa, void *buf)
{
    extern __shared__ char smem_raw[];
    cx<double> *s = reinterpret_cast<cx<double> *>(smem_raw);
    cx<double> *g = (cx<double> *)buf;
    for (int n = threadIdx.x; n < ra.L; n += kThreads) s[n] = g[n];
    __syncthreads();
    fft_lds<double, 16>(s, ra, 1, 1, ra.L, false, (const Tw<double> *)twa);
    for (int n = threadIdx.x; n < ra.L; n += kThreads) g[n] = s[n];
}

// ---------------------------------------------------------------- tables
// natural-order spectrum -> schedule layout (transposed: position k1 L2 + k2
// holds xi = k1 + L1 k2), scaled, complex double
__global__ void k_permute(cx<double> *dst, const cx<double> *src, int64_t L, int L1, int L2,
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
        dst[pos] = {z.x * scale, z.y * scale};
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

// kinetic multipliers per squared norm m: exp(-i kin m) * scale, angle reduced in FP64
__global__ void k_ktab(double *dst, int64_t count, double kin, double scale)
{
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < count;
         m += (int64_t)gridDim.x * blockDim.x) {
        double c, s;
        expm_i(kin * (double)m, c, s);
        dst[2 * m] = c * scale;
        dst[2 * m + 1] = s * scale;
    }
}

// one kinetic table per problem of a batch (blockIdx.y)
__global__ void k_ktab_multi(const KtabDesc *d)
{
    const KtabDesc q = d[blockIdx.y];
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < q.count;
         m += (int64_t)gridDim.x * blockDim.x) {
        double c, s;
        expm_i(q.kin * (double)m, c, s);
        q.dst[2 * m] = c * q.scale;
        q.dst[2 * m + 1] = s * q.scale;
    }
}

// conj(K_xi) = conj(ktab[s[xi]]) for every key xi < N, complex double
__global__ void k_conv_input(cx<double> *dst, const int32_t *s, const double *ktab, int64_t N)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int m = s[n];
        dst[n] = {ktab[2 * m], -ktab[2 * m + 1]};
    }
}

// zero-padded embedding of a length-N cyclic kernel into length L >= 2N-1:
// g_j = conj(src_j) scale for j < N, g_{L-j} = conj(src_{N-j}) scale for
// 0 < j < N, zero elsewhere
__global__ void k_conv_embed(cx<double> *g, const cx<double> *src, int64_t N, int64_t L, double scale)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < L; j += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = -1;
        if (j < N) m = j;
        else if (j > L - N) m = N - (L - j);
        cx<double> z = {0.0, 0.0};
        if (m >= 0) z = {src[m].x * scale, -src[m].y * scale};
        g[j] = z;
    }
}

// the convolution spectrum of a complex64 run, rounded once to complex float
// (count complex entries)
__global__ void k_spectrum_f32(cx<float> *dst, const cx<double> *src, int64_t count)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < count;
         j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = {(float)src[j].x, (float)src[j].y};
}

// per-point multiplier exp(-i phase v[n]) in the run's precision (complex
// double, or rounded once to complex float), angle formed and reduced in FP64
template <typename T>
__global__ void k_phase_table(cx<T> *dst, const double *v, int64_t v_bs, int nv, int64_t N, double phase)
{
    const int b = blockIdx.y;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        double c, s;
        expm_i(phase * v[b * v_bs + n], c, s);
        dst[b * N + n] = {(T)c, (T)s};
    }
}

// per-block partial sums of one state (blockIdx.y), fixed order:
//   p[0] = sum |x_i|^2 * (w ? w[i] : 1),  p[1] = sum |x_i|^2 * vw[i] (vw optional)
constexpr int kSumBlocks = 256;

template <typename T>
__global__ void __launch_bounds__(256) k_sums(const cx<T> *x, int64_t x_bs, int64_t count, const int32_t *w,
                                              const double *vw, int64_t vw_bs, double *partial)
{
    __shared__ double red[2][256];
    const int64_t b = blockIdx.y;
    const cx<T> *xb = x + b * x_bs;
    const double *vb = vw ? vw + b * vw_bs : nullptr;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const cx<T> z = xb[i];
        const double a2 = (double)z.x * (double)z.x + (double)z.y * (double)z.y;
        s0 += w ? a2 * (double)w[i] : a2;
        if (vb) s1 += a2 * vb[i];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *pb = partial + (b * gridDim.x + blockIdx.x) * 2;
        pb[0] = red[0][0];
        pb[1] = red[1][0];
    }
}

// (norm^2, energy) per state from the point sums (|u|^2, v|u|^2) and the
// spectral sum (s |U|^2, scaled by kscale)
__global__ void k_diag_finish(const double *pp, const double *ps, int nblk, int batch, int64_t N, double gamma,
                              double kscale, double *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double n2 = 0.0, pe = 0.0, ke = 0.0;
    for (int i = 0; i < nblk; ++i) {
        n2 += pp[(b * nblk + i) * 2];
        pe += pp[(b * nblk + i) * 2 + 1];
        ke += ps[(b * nblk + i) * 2];
    }
    const double pi = 3.14159265358979323846;
    out[2 * b] = n2 / (double)N;
    out[2 * b + 1] = (2.0 * pi * pi * gamma * ke * kscale + pe / gamma) / (double)N;
}

// Projection sums of one batch item: sum over keys of |ghat|^2 and of
// |ghat - scale x|^2, where x is the lattice DFT of the point values at
// position pos and ghat the caller's coefficient of the key at pos (key =
// pos, or k1 + L1 k2 for the transposed layout pos = k1 L2 + k2)
template <typename T>
__global__ void __launch_bounds__(256) k_proj_sums(const cx<T> *x, int64_t x_bs, int64_t count, double scale,
                                                   int transposed, int L1, int L2, const double *ghat,
                                                   int64_t g_bs, double *partial)
{
    __shared__ double red[2][256];
    const int64_t b = blockIdx.y;
    const cx<T> *xb = x + b * x_bs;
    const double *gb = ghat + 2 * b * g_bs;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t key = i;
        if (transposed) {
            const int64_t k1 = i / L2;
            key = k1 + (int64_t)L1 * (i - k1 * L2);
        }
        const double gr = gb[2 * key], gi = gb[2 * key + 1];
        const cx<T> z = xb[i];
        const double dr = gr - scale * (double)z.x, di = gi - scale * (double)z.y;
        s0 += gr * gr + gi * gi;
        s1 += dr * dr + di * di;
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *pb = partial + (b * gridDim.x + blockIdx.x) * 2;
        pb[0] = red[0][0];
        pb[1] = red[1][0];
    }
}

__global__ void k_proj_finish(const double *partial, int nblk, int batch, double *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < nblk; ++i) {
        s0 += partial[(b * nblk + i) * 2];
        s1 += partial[(b * nblk + i) * 2 + 1];
    }
    out[2 * b] = s0;
    out[2 * b + 1] = s1;
}

// per-step sums of a run: block (j, b) adds the PT tile partials of slot j
// (step j0 + j) of state b in a fixed order and writes the norm^2 and the
// potential energy of that step
__global__ void __launch_bounds__(256) k_step_sums_finish(const double *part, int PT, int batch, int64_t j0,
                                                          int64_t steps, double inv_n, double inv_gn,
                                                          double *hist)
{
    const int64_t j = blockIdx.x;
    const int b = blockIdx.y;
    const double *pb = part + ((size_t)j * batch + b) * (size_t)PT * 2;
    double s1 = 0.0, s2 = 0.0;
    for (int t = threadIdx.x; t < PT; t += 256) {
        s1 += pb[2 * t];
        s2 += pb[2 * t + 1];
    }
    block_sum2<256>(s1, s2);
    if (threadIdx.x == 0) {
        double *h = hist + ((size_t)b * (steps + 1) + j0 + j) * 2;
        h[0] = s1 * inv_n;
        h[1] = s2 * inv_gn;
    }
}

// a fill kernel instead of a memset, so that the zeroing can sit in a
// captured graph
__global__ void k_zero(double *dst, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0.0;
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

// launch with the kernel class's timing events when timing is enabled
template <typename K, typename... A>
static int timed_launch(int kind, K kernel, dim3 grid, dim3 block, size_t lds, void *stream, A... args)
{
    void *e0 = nullptr, *e1 = nullptr;
    timing_events(kind, &e0, &e1);
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, block, lds, (hipStream_t)stream, (hipEvent_t)e0, (hipEvent_t)e1, 0,
                              args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, (hipStream_t)stream, args...);
    return (int)hipGetLastError();
}

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
    const int lim = kMaxDynLds;
    hipFuncSetAttribute((const void *)k_col<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_col<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_col<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_col<double, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row<float, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row<double, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_resident<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_resident<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_col_multi<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_col_multi<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row_multi<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_row_multi<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_resident_multi<float, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipFuncSetAttribute((const void *)k_resident_multi<double, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    hipGetLastError();
    return 0;
}

int launch_col(int prec, const Sched &s, const ColArgs &a, int batch, void *stream)
{
    const int var = col_variant_of(s, batch);
    if (var > 0) {
        ColArgs f = a;
        f.wt = cache_resident(s, esize(prec), batch) ? 1 : 0;
        const int r = a.adjoint ? launch_col_fast_adjoint(prec, var, f, batch, stream)
                                : launch_col_fast(prec, var, f, batch, stream);
        if (r >= 0) return r;
    }
    const int nvec = a.adjoint ? 2 : 1;
    const size_t lds = (size_t)a.L1 * a.C * nvec * esize(prec);
    dim3 grid(a.ntiles, batch);
    if (a.adjoint && (int64_t)a.L1 * a.C * 2 > kTileElems) {  // state and cotangent: up to 2 x 4096 elements
        if (prec == LT_C128)
            return timed_launch(LT_KIND_COLUMN, k_col<double, 32>, grid, dim3(kThreads), lds, stream, a);
        return timed_launch(LT_KIND_COLUMN, k_col<float, 32>, grid, dim3(kThreads), lds, stream, a);
    }
    if (prec == LT_C128)
        return timed_launch(LT_KIND_COLUMN, k_col<double, 16>, grid, dim3(kThreads), lds, stream, a);
    return timed_launch(LT_KIND_COLUMN, k_col<float, 16>, grid, dim3(kThreads), lds, stream, a);
}

int launch_row(int prec, const Sched &s, const RowArgs &a, int batch, void *stream)
{
    const int var = row_variant_of(s, batch);
    if (var > 0 && !a.fft_only) {
        RowArgs f = a;
        f.wt = cache_resident(s, esize(prec), batch) ? 1 : 0;
        const int r = launch_row_fast(prec, var, f, batch, stream);
        if (r >= 0) return r;
    }
    const size_t lds = (size_t)a.rows * a.L2 * esize(prec);
    dim3 grid(a.nblk, batch);
    if ((int64_t)a.rows * a.L2 > kTileElems) {  // one row of up to kWideRow points
        if (prec == LT_C128)
            return timed_launch(LT_KIND_ROW, k_row<double, 32>, grid, dim3(kThreads), lds, stream, a);
        return timed_launch(LT_KIND_ROW, k_row<float, 32>, grid, dim3(kThreads), lds, stream, a);
    }
    if (prec == LT_C128)
        return timed_launch(LT_KIND_ROW, k_row<double, 16>, grid, dim3(kThreads), lds, stream, a);
    return timed_launch(LT_KIND_ROW, k_row<float, 16>, grid, dim3(kThreads), lds, stream, a);
}

int launch_resident(int prec, const Sched &s, const ResArgs &a, int batch, void *stream)
{
    const size_t lds = (size_t)a.L * esize(prec);
    (void)s;
    if (prec == LT_C128)
        return timed_launch(LT_KIND_RESIDENT, k_resident<double, 16>, dim3(batch), dim3(kThreads), lds, stream, a);
    return timed_launch(LT_KIND_RESIDENT, k_resident<float, 16>, dim3(batch), dim3(kThreads), lds, stream, a);
}

int launch_col_multi(int prec, const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks,
                     int off, int64_t g, size_t lds, void *stream)
{
    const int grid = (nblocks + 7) / 8 * 8;
    if (prec == LT_C128)
        return timed_launch(LT_KIND_COLUMN, k_col_multi<double, 16>, dim3(grid), dim3(kThreads), lds, stream,
                            d, idx, start, nmem, nblocks, off, g);
    return timed_launch(LT_KIND_COLUMN, k_col_multi<float, 16>, dim3(grid), dim3(kThreads), lds, stream, d,
                        idx, start, nmem, nblocks, off, g);
}

int launch_row_multi(int prec, const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks,
                     int off, int64_t g, size_t lds, void *stream)
{
    if (prec == LT_C128)
        return timed_launch(LT_KIND_ROW, k_row_multi<double, 16>, dim3(nblocks), dim3(kThreads), lds, stream,
                            d, idx, start, nmem, off, g);
    return timed_launch(LT_KIND_ROW, k_row_multi<float, 16>, dim3(nblocks), dim3(kThreads), lds, stream, d, idx,
                        start, nmem, off, g);
}

int launch_ktab_multi(const KtabDesc *d, int count, int64_t max_len, void *stream)
{
    if (count <= 0) return 0;
    int gx = grid1d(max_len);
    if (gx > 64) gx = 64;
    hipLaunchKernelGGL(k_ktab_multi, dim3(gx, count), dim3(256), 0, (hipStream_t)stream, d);
    return (int)hipGetLastError();
}

int launch_resident_multi(int prec, const ResArgs *d, int ninst, size_t lds, void *stream)
{
    if (prec == LT_C128)
        return timed_launch(LT_KIND_RESIDENT, k_resident_multi<double, 16>, dim3(ninst), dim3(kThreads), lds,
                            stream, d);
    return timed_launch(LT_KIND_RESIDENT, k_resident_multi<float, 16>, dim3(ninst), dim3(kThreads), lds, stream,
                        d);
}

int launch_step_sums_finish(const double *part, int PT, int batch, int64_t j0, int64_t count, int64_t steps,
                            double inv_n, double inv_gn, double *hist, void *stream)
{
    if (count <= 0) return 0;
    hipLaunchKernelGGL(k_step_sums_finish, dim3((unsigned)count, batch), dim3(256), 0, (hipStream_t)stream, part, PT,
                       batch, j0, steps, inv_n, inv_gn, hist);
    return (int)hipGetLastError();
}

int launch_zero(double *dst, int64_t count, void *stream)
{
    if (count <= 0) return 0;
    hipLaunchKernelGGL(k_zero, dim3(grid1d(count) > 1024 ? 1024 : grid1d(count)), dim3(256), 0, (hipStream_t)stream,
                       dst, count);
    return (int)hipGetLastError();
}

int launch_fft_single(const Radices &ra, const void *twa, void *buf, int64_t L, void *stream)
{
    hipLaunchKernelGGL(k_fft_single, dim3(1), dim3(kThreads), (size_t)L * 16, (hipStream_t)stream, ra,
                       twa, buf);
    return (int)hipGetLastError();
}

int launch_permute_c128(void *dst, const void *src, int64_t L, int L1, int L2, int transposed,
                        double scale, void *stream)
{
    hipLaunchKernelGGL(k_permute, dim3(grid1d(L)), dim3(256), 0, (hipStream_t)stream, (cx<double> *)dst,
                       (const cx<double> *)src, L, L1, L2, transposed, scale);
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

int launch_ktab(double *dst, int64_t count, double kin, double scale, void *stream)
{
    hipLaunchKernelGGL(k_ktab, dim3(grid1d(count)), dim3(256), 0, (hipStream_t)stream, dst, count, kin,
                       scale);
    return (int)hipGetLastError();
}

int launch_conv_input(void *dst, const int32_t *s, const double *ktab, int64_t N, void *stream)
{
    hipLaunchKernelGGL(k_conv_input, dim3(grid1d(N)), dim3(256), 0, (hipStream_t)stream, (cx<double> *)dst, s,
                       ktab, N);
    return (int)hipGetLastError();
}

int launch_conv_embed(void *g, const void *src, int64_t N, int64_t L, double scale, void *stream)
{
    hipLaunchKernelGGL(k_conv_embed, dim3(grid1d(L)), dim3(256), 0, (hipStream_t)stream, (cx<double> *)g,
                       (const cx<double> *)src, N, L, scale);
    return (int)hipGetLastError();
}

int launch_spectrum_f32(void *dst, const void *src, int64_t count, void *stream)
{
    hipLaunchKernelGGL(k_spectrum_f32, dim3(grid1d(count) > 2048 ? 2048 : grid1d(count)), dim3(256), 0,
                       (hipStream_t)stream, (cx<float> *)dst, (const cx<double> *)src, count);
    return (int)hipGetLastError();
}

int launch_phase_table(int prec, void *dst, const double *v, int64_t v_bs, int nv, int64_t N, double phase,
                       void *stream)
{
    dim3 grid(grid1d(N) > 2048 ? 2048 : grid1d(N), nv);
    if (prec == LT_C128)
        hipLaunchKernelGGL(k_phase_table<double>, grid, dim3(256), 0, (hipStream_t)stream, (cx<double> *)dst, v,
                           v_bs, nv, N, phase);
    else
        hipLaunchKernelGGL(k_phase_table<float>, grid, dim3(256), 0, (hipStream_t)stream, (cx<float> *)dst, v,
                           v_bs, nv, N, phase);
    return (int)hipGetLastError();
}

int diag_partials() { return kSumBlocks; }

int launch_sums(int prec, const void *x, int64_t x_bs, int64_t count, int batch, const int32_t *w,
                const double *vw, int64_t vw_bs, double *partial, void *stream)
{
    dim3 grid(kSumBlocks, batch);
    if (prec == LT_C128)
        hipLaunchKernelGGL(k_sums<double>, grid, dim3(256), 0, (hipStream_t)stream, (const cx<double> *)x, x_bs,
                           count, w, vw, vw_bs, partial);
    else
        hipLaunchKernelGGL(k_sums<float>, grid, dim3(256), 0, (hipStream_t)stream, (const cx<float> *)x, x_bs,
                           count, w, vw, vw_bs, partial);
    return (int)hipGetLastError();
}

int launch_diag_finish(const double *pp, const double *ps, int batch, int64_t N, double gamma, double kscale,
                       double *out, void *stream)
{
    hipLaunchKernelGGL(k_diag_finish, dim3((batch + 127) / 128), dim3(128), 0, (hipStream_t)stream, pp, ps,
                       kSumBlocks, batch, N, gamma, kscale, out);
    return (int)hipGetLastError();
}

int launch_proj_sums(int prec, const void *x, int64_t x_bs, int64_t count, int batch, double scale, int transposed,
                     int L1, int L2, const double *ghat, int64_t g_bs, double *partial, double *out, void *stream)
{
    dim3 grid(kSumBlocks, batch);
    if (prec == LT_C128)
        hipLaunchKernelGGL(k_proj_sums<double>, grid, dim3(256), 0, (hipStream_t)stream, (const cx<double> *)x,
                           x_bs, count, scale, transposed, L1, L2, ghat, g_bs, partial);
    else
        hipLaunchKernelGGL(k_proj_sums<float>, grid, dim3(256), 0, (hipStream_t)stream, (const cx<float> *)x,
                           x_bs, count, scale, transposed, L1, L2, ghat, g_bs, partial);
    const int e = (int)hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL(k_proj_finish, dim3((batch + 127) / 128), dim3(128), 0, (hipStream_t)stream, partial,
                       kSumBlocks, batch, out);
    return (int)hipGetLastError();
}

// dst[b][c][r] = src[b][r][c] for a batch of rows x cols matrices, through
// 32 x 32 tiles in LDS (rows of the tile read and written contiguously)
struct alignas(16) B16 {
    double x, y;
};
template <typename E>
__global__ void __launch_bounds__(256) k_transpose(E *dst, const E *src, int rows, int cols, int64_t dst_bs,
                                                   int64_t src_bs)
{
    __shared__ E t[32][33];
    const E *sb = src + (int64_t)blockIdx.z * src_bs;
    E *db = dst + (int64_t)blockIdx.z * dst_bs;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) t[i][tx] = sb[(int64_t)r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (r < rows && c < cols) db[(int64_t)c * rows + r] = t[tx][i];
    }
}

int launch_transpose(int esize, void *dst, const void *src, int batch, int rows, int cols, int64_t dst_bs,
                     int64_t src_bs, void *stream)
{
    if (batch < 1 || rows < 1 || cols < 1 || (esize != 8 && esize != 16)) return (int)hipErrorInvalidValue;
    // the batch runs along the grid's z, in chunks of at most 65535
    for (int b0 = 0; b0 < batch; b0 += 65535) {
        const dim3 grid((cols + 31) / 32, (rows + 31) / 32, std::min(65535, batch - b0));
        const size_t d0 = (size_t)b0 * dst_bs * esize, s0 = (size_t)b0 * src_bs * esize;
        if (esize == 16)
            hipLaunchKernelGGL(k_transpose<B16>, grid, dim3(256), 0, (hipStream_t)stream,
                               (B16 *)((char *)dst + d0), (const B16 *)((const char *)src + s0), rows, cols,
                               dst_bs, src_bs);
        else
            hipLaunchKernelGGL(k_transpose<uint64_t>, grid, dim3(256), 0, (hipStream_t)stream,
                               (uint64_t *)((char *)dst + d0), (const uint64_t *)((const char *)src + s0), rows,
                               cols, dst_bs, src_bs);
        const int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

int launch_reduce_batch(double *dst, const double *src, int64_t N, int batch, void *stream)
{
    hipLaunchKernelGGL(k_reduce_batch, dim3(grid1d(N)), dim3(256), 0, (hipStream_t)stream, dst, src,
                       N, batch);
    return (int)hipGetLastError();
}

}  // namespace lt
