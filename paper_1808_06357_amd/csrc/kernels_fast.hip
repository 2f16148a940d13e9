// Register-staged column / row passes for the power-of-two lengths 64..4096
// (mixed radices 2..16 with equal first and last radix).
//
// Compared with the general kernels:
//  * each thread owns E elements; every stage is E / R radix-R butterflies
//    per thread, fully unrolled at compile time;
//  * the first stage reads global memory straight into registers and the last
//    stage's outputs stay in registers: the column pass goes
//    [global -> inverse DFT -> point-domain phase -> forward DFT -> global] and
//    the row pass [global -> DFT -> spectral multiplier -> inverse DFT ->
//    global] with LDS used only for the NS-1 exchanges inside each DFT;
//  * the state and the per-element tables are read and written through
//    buffer resources: one 32-bit lane offset per butterfly group plus a
//    wave-uniform offset per radix element, so addresses cost few registers
//    and every load of a tile is issued before the first use; the four-step
//    twiddle base and step of a group are formed once and reused for the
//    forward pass;
//  * LDS indices are padded (one slot every 16 elements) so the strided
//    Stockham writes do not pile onto a few banks;
//  * column tiles are remapped so that neighbouring tiles, which share cache
//    lines, run on the same XCD (workgroups are dealt round-robin to the 8
//    XCDs, each with its own L2).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "device.h"
#include "lt_internal.h"

namespace lt {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Buffer-resource access (gfx9 raw buffers): a per-lane 32-bit byte offset
// plus a wave-uniform byte offset held in a scalar register, so that the
// addresses of a thread's R elements cost one vector register instead of R
// 64-bit pairs.  num_records bounds every access (out-of-range loads read 0,
// stores are dropped); offsets here always stay inside the buffer.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ cx<T> bload(rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ cx<float> bload<float>(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ cx<double> bload<double>(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// State stores: SA is the instruction's cache-policy operand.  A pass whose
// working set fits the Infinity Cache stores with the device-scope coherence
// bit (kWriteThrough, sc1): the next pass, on every XCD, reads what this one
// writes, and a write-back L2 would hold the dirty lines until the release at
// the end of the kernel.  Measured on the 2^21-point convolution (67 MB per
// pass): row pass 13.8 -> 12.3 us (complex64), 16.6 -> 15.7 us (complex128),
// rank-2 2^20 points 4.7e10 -> 6.3e10 pt-steps/s.  Beyond the cache
// (working sets of 270-450 MB) the plain write-back stores are 2-4 % faster,
// so launches choose by their working set.  Streaming (nt) stores or loads
// were slower in both regimes.
constexpr int kWriteThrough = 16;

template <int SA = 0>
__device__ __forceinline__ void bstore(cx<float> x, rsrc_t r, uint32_t voff, uint32_t soff)
{
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, voff, soff, SA);
}
template <int SA = 0>
__device__ __forceinline__ void bstore(cx<double> x, rsrc_t r, uint32_t voff, uint32_t soff)
{
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, x), r, voff, soff, SA);
}

__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// Entry of the per-point table of the merged potential step exp(-i phase v):
// complex64 runs keep it rounded once to complex float (the phase itself is
// formed and reduced in double), complex128 runs in complex double.  Either
// way one entry is as wide as one state element, so it sits at the element's
// own byte offset.
template <typename T>
struct PTabT;
template <>
struct PTabT<float> {
    using type = cx<float>;
};
template <>
struct PTabT<double> {
    using type = Tw<double>;
};
template <typename T>
using PTab = typename PTabT<T>::type;

template <typename T>
__device__ __forceinline__ PTab<T> pload(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ PTab<float> pload<float>(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ PTab<double> pload<double>(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(Tw<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ cx<float> ptmul(cx<float> a, cx<float> t)
{
    return {a.x * t.x - a.y * t.y, a.x * t.y + a.y * t.x};
}
__device__ __forceinline__ cx<double> ptmul(cx<double> a, const Tw<double> &t) { return twmul(a, t); }
__device__ __forceinline__ cx<double> pt_d(cx<float> t) { return {(double)t.x, (double)t.y}; }
__device__ __forceinline__ cx<double> pt_d(const Tw<double> &t) { return t.w; }

// x[r] *= w^r for r = 1..R-1, w in double: two running powers (odd and even
// exponents, each stepped by w^2), multiplied and applied in turn, so that
// only three complex doubles stay live and the two chains overlap.  Each
// power is at most ~R/2 double roundings deep, far below the rounding of the
// data.  The products are formed and applied in double even for complex64
// data: float twiddles carry a fixed rounding error that repeats every step
// and adds up coherently (measured: 1.7e-4 relative after 1000 steps of the
// 2^21-point convolution, against 4.8e-6 with the double products).
template <typename T, int R>
__device__ __forceinline__ void apply_powers(cx<T> *x, double wr, double wi)
{
    const double qr = wr * wr - wi * wi, qi = 2.0 * wr * wi;  // w^2
    double ar = wr, ai = wi, br = qr, bi = qi;                // w^1, w^2
#pragma unroll
    for (int r = 1; r < R; r += 2) {
        x[r] = cmul_d(x[r], ar, ai);
        if (r + 1 < R) x[r + 1] = cmul_d(x[r + 1], br, bi);
        if (r + 2 < R) {
            const double nr = ar * qr - ai * qi, ni = ar * qi + ai * qr;
            ar = nr;
            ai = ni;
        }
        if (r + 3 < R) {
            const double nr = br * qr - bi * qi, ni = br * qi + bi * qr;
            br = nr;
            bi = ni;
        }
    }
}

// x[r] *= b s^r for r = 0..R-1 (a four-step twiddle series), in double, with
// the same two-chain evaluation as apply_powers
template <typename T, int R>
__device__ __forceinline__ void apply_series(cx<T> *x, cx<double> b, cx<double> st)
{
    const double qr = st.x * st.x - st.y * st.y, qi = 2.0 * st.x * st.y;  // s^2
    double ar = b.x, ai = b.y;                                             // b s^0
    double br = b.x * st.x - b.y * st.y, bi = b.x * st.y + b.y * st.x;     // b s^1
#pragma unroll
    for (int r = 0; r < R; r += 2) {
        x[r] = cmul_d(x[r], ar, ai);
        if (r + 1 < R) x[r + 1] = cmul_d(x[r + 1], br, bi);
        if (r + 2 < R) {
            const double nr = ar * qr - ai * qi, ni = ar * qi + ai * qr;
            ar = nr;
            ai = ni;
        }
        if (r + 3 < R) {
            const double nr = br * qr - bi * qi, ni = br * qi + bi * qr;
            br = nr;
            bi = ni;
        }
    }
}

// Stockham DFT over a tile of NT*E elements = SEQ sequences of length
// L = R_0 R_1 ... R_{NS-1} (radices Rs, first and last equal).  COLS: element
// e of sequence q at e*SEQ + q (interleaved columns); otherwise at q*L + e
// (contiguous rows).  In stage s butterfly bf = tid + j*NT handles sequence q,
// index t < L/R_s and the elements t + r L/R_s; the thread's E elements sit in
// x[j R_s + r].  On entry x holds the first stage's inputs, on exit the last
// stage's outputs (the same positions, since the two radices agree).  The
// stage twiddles W_{Ns R_s}^{(t mod Ns) r} are powers of one base per stage
// and butterfly; the bases are loaded once (load_bases) and the powers formed
// in double (apply_powers).
template <int... Rs>
struct Radix {
    static constexpr int n = sizeof...(Rs);
    static constexpr int v[n] = {Rs...};
    static constexpr int prod = (1 * ... * Rs);
    static constexpr int min()
    {
        int m = v[0];
        for (int i = 1; i < n; ++i) m = v[i] < m ? v[i] : m;
        return m;
    }
    static constexpr int before(int st)
    {
        int p = 1;
        for (int i = 0; i < st; ++i) p *= v[i];
        return p;
    }
};

template <typename T, int E, int NT, bool COLS, int... Rs>
struct Fft {
    using RL = Radix<Rs...>;
    static constexpr int NS = RL::n;
    static constexpr int L = RL::prod;
    static constexpr int R = RL::v[0];
    static constexpr int TILE = NT * E;
    static constexpr int SEQ = TILE / L;
    static constexpr int J = E / R;
    static constexpr int BPS = L / R;
    static constexpr int NB = NS > 1 ? NS - 1 : 1;
    static constexpr int MAXJ = E / RL::min();
    static_assert(RL::v[0] == RL::v[NS - 1], "first and last radix must agree");
    static_assert(((E % Rs == 0) && ...) && TILE % L == 0, "tile must hold whole sequences");

    struct Bases {
        double r[NB][MAXJ], i[NB][MAXJ];
    };

    static __device__ __forceinline__ int qs(int bf, int bps) { return COLS ? bf % SEQ : bf / bps; }
    static __device__ __forceinline__ int ts(int bf, int bps) { return COLS ? bf / SEQ : bf % bps; }
    static __device__ __forceinline__ int q_of(int bf) { return qs(bf, BPS); }
    static __device__ __forceinline__ int t_of(int bf) { return ts(bf, BPS); }
    static __device__ __forceinline__ int addr(int q, int e) { return pidx(COLS ? e * SEQ + q : q * L + e); }

    template <int ST>
    static __device__ __forceinline__ void bases_from(Bases &B, const Tw<T> *__restrict__ tw)
    {
        if constexpr (ST < NS) {
            constexpr int Rc = RL::v[ST], Jc = E / Rc, BPSc = L / Rc, Ns = RL::before(ST);
            constexpr int twstep = L / (Ns * Rc);
#pragma unroll
            for (int j = 0; j < Jc; ++j) {
                const int t = ts(threadIdx.x + j * NT, BPSc);
                const cx<double> w = tw_d(tw[(t % Ns) * twstep]);
                B.r[ST - 1][j] = w.x;
                B.i[ST - 1][j] = w.y;
            }
            bases_from<ST + 1>(B, tw);
        }
    }

    static __device__ __forceinline__ void load_bases(Bases &B, const Tw<T> *__restrict__ tw)
    {
        bases_from<1>(B, tw);
    }

    template <int ST>
    static __device__ __forceinline__ void stages_from(cx<T> (&x)[E], cx<T> *s, const Bases &B, bool sync_first)
    {
        if constexpr (ST < NS) {
            constexpr int Rp = RL::v[ST - 1], Jp = E / Rp, BPSp = L / Rp, Nsp = RL::before(ST - 1);
            constexpr int Rc = RL::v[ST], Jc = E / Rc, BPSc = L / Rc;
            if (ST > 1 || sync_first) __syncthreads();
#pragma unroll
            for (int j = 0; j < Jp; ++j) {
                const int bf = threadIdx.x + j * NT;
                const int q = qs(bf, BPSp), t = ts(bf, BPSp);
                const int jj = t % Nsp;
                const int ob = (t - jj) * Rp + jj;
#pragma unroll
                for (int r = 0; r < Rp; ++r) s[addr(q, ob + r * Nsp)] = x[j * Rp + r];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < Jc; ++j) {
                const int bf = threadIdx.x + j * NT;
                const int q = qs(bf, BPSc), t = ts(bf, BPSc);
#pragma unroll
                for (int r = 0; r < Rc; ++r) x[j * Rc + r] = s[addr(q, t + r * BPSc)];
                apply_powers<T, Rc>(&x[j * Rc], B.r[ST - 1][j], B.i[ST - 1][j]);
                Dft<T, Rc>::run(&x[j * Rc]);
            }
            stages_from<ST + 1>(x, s, B, sync_first);
        }
    }

    static __device__ __forceinline__ void run(cx<T> (&x)[E], cx<T> *s, const Bases &B, bool sync_first)
    {
#pragma unroll
        for (int j = 0; j < J; ++j) Dft<T, R>::run(&x[j * R]);
        stages_from<1>(x, s, B, sync_first);
    }
};

__device__ __forceinline__ int xcd_tile(int bid, int n)
{
    if (n % 8) return bid;
    return (bid % 8) * (n / 8) + bid / 8;
}

// Four-step twiddles W_L^{n2 k} for k = t + r*BPS, r = 0..R-1: base
// W^{n2 t} and step W^{n2 BPS} from the two-level tables, in double
// (apply_series forms and applies the series)
__device__ __forceinline__ void tw4_base_step(cx<double> &b, cx<double> &st, int n2, int t, int BPS, int L2,
                                              const double *hi, const double *lo)
{
    const cx<double> one = {1.0, 0.0};
    b = tw4mul(one, n2, t, L2, hi, lo);
    st = tw4mul(one, n2, BPS, L2, hi, lo);
}

// Registers of one column tile between its loads and its transforms: the
// tile's elements, their byte offsets, and (complex64 table steps) the table
// entries of the first butterfly group.
template <typename T, int E, int J, int R, bool PRE, bool PV>
struct ColTile {
    cx<T> v[E];
    uint32_t voff[J];
    PTab<T> pre[PRE ? R : 1];
    double sv[PV ? E : 1];  // v of every element for the step's sums (MID 8, eight elements or fewer)
};

// MID 8 with at most eight elements per thread: v of the tile's elements is
// loaded with the state (its latency then hides behind the inverse DFT
// instead of stalling the sums between the transforms)
template <int MID, int E>
constexpr bool col_prefetch_v()
{
    return MID == 8 && E <= 8;
}

// complex64 merged potential step: with two or more butterfly groups per
// thread, or several tiles per workgroup, the table entries of the first
// group are loaded with the state (halving the burst of table loads after
// the inverse DFT), the rest after the inverse DFT.  Not with the step's
// sums and two groups per thread: holding those entries through the sums
// spills.
template <typename T, int MID, int J, int S>
constexpr bool col_prefetch()
{
    return sizeof(T) == 4 && ((MID == 0 && (J > 1 || S > 1)) || (MID == 8 && J == 1 && S > 1));
}

// Issues every load of column tile `tile` of batch item b: element
// (t + r BPS, c0 + q) sits at byte voff[j] + r * rstep of the state
// (IN: from the run's input vector, whose zero padding n >= Nvalid lies
// beyond its range and reads 0)
template <typename T, int E, int NT, bool PRE, bool PV, bool IN, int... Rs>
__device__ __forceinline__ void colf_load(const ColArgs &a, int tile, int64_t b,
                                          ColTile<T, E, Fft<T, E, NT, true, Rs...>::J, Fft<T, E, NT, true, Rs...>::R, PRE, PV> &X)
{
    using F = Fft<T, E, NT, true, Rs...>;
    constexpr int C = F::SEQ, J = F::J, R = F::R, BPS = F::BPS, L1 = F::L;
    const int L2 = a.L2;
    const int c0 = tile * C;
    const cx<T> *src = IN ? (const cx<T> *)a.in + b * a.in_bs : (const cx<T> *)a.buf + b * a.buf_bs;
    const rsrc_t rb = make_rsrc(src, (IN ? a.Nvalid : (int64_t)L1 * L2) * (int64_t)sizeof(cx<T>));
    const uint32_t rstep = (uint32_t)BPS * (uint32_t)L2 * (uint32_t)sizeof(cx<T>);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int bf = threadIdx.x + j * NT;
        X.voff[j] = ((uint32_t)F::t_of(bf) * (uint32_t)L2 + (uint32_t)(c0 + F::q_of(bf))) * (uint32_t)sizeof(cx<T>);
#pragma unroll
        for (int r = 0; r < R; ++r) X.v[j * R + r] = bload<T>(rb, X.voff[j], r * rstep);
    }
    if constexpr (PV) {
        // v at the element's offset scaled to 8 bytes; the zero padding
        // (n >= Nvalid) lies beyond the buffer's range and reads 0
        const rsrc_t rv = make_rsrc(a.sum_v + b * a.v_bs, a.Nvalid * (int64_t)sizeof(double));
        constexpr uint32_t vdiv = (uint32_t)(sizeof(cx<T>) / sizeof(double));
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                X.sv[j * R + r] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(rv, (X.voff[j] + r * rstep) / vdiv, 0, 0));
        }
    }
    if constexpr (PRE) {
        const rsrc_t rp = make_rsrc((const PTab<T> *)a.ptab + b * a.ptab_bs, a.Nvalid * (int64_t)sizeof(PTab<T>));
#pragma unroll
        for (int r = 0; r < R; ++r) X.pre[r] = pload<T>(rp, X.voff[0] + r * rstep);
    }
}

// The step's sums of |u|^2 and v |u|^2 over column tile `tile` of batch item
// b, from the tile's values x in registers (|x| = |u| at a step boundary): v
// of each element at the element's offset scaled to 8 bytes (or from sv, when
// it was loaded with the state); the zero padding (n >= Nvalid) is masked by
// its offset.  One partial pair per tile.
template <typename T, int E, int NT, int J, int R, bool PV>
__device__ __forceinline__ void tile_sums(const ColArgs &a, int tile, int64_t b, const cx<T> (&v)[E],
                                          const uint32_t (&voff)[J], uint32_t rstep, const double *sv)
{
    const rsrc_t rv = make_rsrc(a.sum_v + b * a.v_bs, a.Nvalid * (int64_t)sizeof(double));
    constexpr uint32_t vdiv = (uint32_t)(sizeof(cx<T>) / sizeof(double));
    const uint32_t lim = (uint32_t)a.Nvalid * (uint32_t)sizeof(cx<T>);
    // v is loaded in chunks of at most eight elements (sixteen registers in
    // flight), which keeps the 16-element geometries from spilling; the
    // accumulation order is that of the elements either way
    constexpr int CH = R > 8 ? 8 : R;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
        for (int r0 = 0; r0 < R; r0 += CH) {
            double vv[CH];
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                if constexpr (PV) vv[r] = sv[j * R + r0 + r];
                else
                    vv[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                           rv, (voff[j] + (r0 + r) * rstep) / vdiv, 0, 0));
            }
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                const cx<T> x = v[j * R + r0 + r];
                const double q2 = voff[j] + (r0 + r) * rstep < lim
                                      ? (double)x.x * (double)x.x + (double)x.y * (double)x.y
                                      : 0.0;
                s1 += q2;
                s2 += vv[r] * q2;
            }
            if constexpr (CH < R) __builtin_amdgcn_sched_barrier(0);
        }
    }
    block_sum2<NT>(s1, s2);
    if (threadIdx.x == 0) {
        double *pb = a.sum_part + ((int64_t)b * a.sum_pt + tile) * 2;
        pb[0] = s1;
        pb[1] = s2;
    }
}

// Steady-state column pass: [inverse column DFT -> point-domain multiplier
// (and chirp-z mask) -> forward column DFT], in place, on column tile `tile`
// of batch item b, whose loads colf_load issued.  MID 0: the merged potential
// step from the per-point table the run built; MID 1: the chirp-z
// kinetic step from the table indexed by the squared norm; MID 2: the merged
// potential step from v in FP64 (runs without a table); MID 3: the angle of
// a time-dependent potential from two fields; MID 7: MID 0 plus the store of
// the step's checkpoint (and the step's sums when asked for); MID 8: MID 0
// plus the step's sums of |u|^2 and v |u|^2.  MID 9: the first pass of a run
// (the half potential step exp(-i phase v) on the input vector, then the
// forward column DFT), MID 10: the last (inverse column DFT, half potential
// step, store to the output vector); both in FP64 from v, with the step's
// sums when asked for.  sync_first: the workgroup used the LDS buffer before
// (a previous tile), so the first write waits for it.
template <typename T, int E, int NT, int MID, bool PRE, bool PV, int SA, int... Rs>
__device__ __forceinline__ void colf_run(const ColArgs &a, int tile, int64_t b, cx<T> *s,
                                         const typename Fft<T, E, NT, true, Rs...>::Bases &B,
                                         ColTile<T, E, Fft<T, E, NT, true, Rs...>::J, Fft<T, E, NT, true, Rs...>::R, PRE, PV> &X,
                                         bool sync_first)
{
    using F = Fft<T, E, NT, true, Rs...>;
    constexpr int C = F::SEQ, J = F::J, R = F::R, BPS = F::BPS, L1 = F::L, TILE = F::TILE;
    const int L2 = a.L2;
    const int c0 = tile * C;
    // MID 10 stores into the output vector; its zero padding (n >= Nvalid)
    // lies beyond that range and is dropped
    cx<T> *dst = MID == 10 ? (cx<T> *)a.out + b * a.out_bs : (cx<T> *)a.buf + b * a.buf_bs;
    const rsrc_t rb = make_rsrc(dst, (MID == 10 ? a.Nvalid : (int64_t)L1 * L2) * (int64_t)sizeof(cx<T>));
    const uint32_t rstep = (uint32_t)BPS * (uint32_t)L2 * (uint32_t)sizeof(cx<T>);
    cx<T>(&v)[E] = X.v;
    const uint32_t(&voff)[J] = X.voff;
    constexpr bool kPreP = PRE;
    // four-step twiddle base and step of each butterfly group: the forward
    // pass at the end multiplies by the same series, so they are kept
    const bool tw = a.twiddle != 0;
    cx<double> tb[J], ts[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        tb[j] = {1.0, 0.0};
        ts[j] = {1.0, 0.0};
    }
    if (tw) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int bf = threadIdx.x + j * NT;
            tw4_base_step(tb[j], ts[j], c0 + F::q_of(bf), F::t_of(bf), BPS, L2, a.tw4hi, a.tw4lo);
        }
    }
    // MID 5: forward DFT only (then the four-step twiddle); MID 6: inverse
    // DFT only (the conjugated twiddle first) -- the inner passes of a
    // three-level transform; MIDs 9 and 10 likewise for a run's first and
    // last passes
    constexpr bool kInv = MID != 5 && MID != 9, kFwd = MID != 6 && MID != 10;
    if constexpr (kInv) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[j * R + r] = conjg(v[j * R + r]);
            if (tw) apply_series<T, R>(&v[j * R], tb[j], ts[j]);
        }
        F::run(v, s, B, sync_first);
    }
    // point-domain multiplier: the table entries of all of this thread's
    // elements are loaded in one batch (one exposed latency), then applied
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (MID == 5) {
        // nothing between the transforms
    } else if constexpr (MID == 6) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = conjg(v[e]);
    } else if constexpr (MID == 0 || MID == 7 || MID == 8) {
        if constexpr (MID == 7) {
            // checkpoint of the state at this step boundary: the lattice value
            // u = x exp(-i ck_phase v) of every valid point, in FP64 like the
            // general pass, stored before the merged step.  The point values
            // go through LDS (free between the two transforms) so that one
            // rolled loop, consecutive lanes on consecutive columns, evaluates
            // the phases without holding them for every element at once.
            __syncthreads();
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int bf = threadIdx.x + j * NT;
                const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
                for (int r = 0; r < R; ++r) s[F::addr(q, t + r * BPS)] = conjg(v[j * R + r]);
            }
            __syncthreads();
            // the same loop forms the step's sums of |u|^2 and v |u|^2 when
            // asked for (|x| = |u| at the boundary)
            const double *cv = a.ck ? a.ck_v + b * a.v_bs : nullptr;
            const double *sv = a.sum_part ? a.sum_v + b * a.v_bs : nullptr;
            cx<T> *ck = a.ck ? (cx<T> *)a.ck + b * a.ck_bs : nullptr;
            double s1 = 0.0, s2 = 0.0;
#pragma unroll 1
            for (int i = threadIdx.x; i < C * L1; i += NT) {
                const int k1 = i / C, q = i - k1 * C;
                const int64_t n = (int64_t)k1 * L2 + c0 + q;
                if (n < a.Nvalid) {
                    const cx<T> x = s[F::addr(q, k1)];
                    if (ck) {
                        double c, sn;
                        expm_i(a.ck_phase * cv[n], c, sn);
                        ck[a.ck_t ? (int64_t)(c0 + q) * L1 + k1 : n] = cmul_d(x, c, sn);
                    }
                    if (sv) {
                        const double q2 = (double)x.x * (double)x.x + (double)x.y * (double)x.y;
                        s1 += q2;
                        s2 += sv[n] * q2;
                    }
                }
            }
            if (sv) {
                block_sum2<NT>(s1, s2);
                if (threadIdx.x == 0) {
                    double *pb = a.sum_part + ((int64_t)b * a.sum_pt + tile) * 2;
                    pb[0] = s1;
                    pb[1] = s2;
                }
            }
        }
        // the values are conjugates of the point values: same modulus
        if constexpr (MID == 8) tile_sums<T, E, NT, J, R, PV>(a, tile, b, v, voff, rstep, X.sv);
        // the merged potential step from the per-point table (one entry as
        // wide as the element, at its offset), every entry of the thread in
        // flight at once.  The whole byte offset sits in the per-lane
        // register, so the buffer's range check reads the entries of the zero
        // padding (n >= Nvalid) as 0, which zeroes those points.
        const rsrc_t rp = make_rsrc((const PTab<T> *)a.ptab + b * a.ptab_bs, a.Nvalid * (int64_t)sizeof(PTab<T>));
        constexpr int j0 = kPreP ? 1 : 0;
        PTab<T> pin[J][R];
#pragma unroll
        for (int j = j0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) pin[j][r] = pload<T>(rp, voff[j] + r * rstep);
        }
        if constexpr (kPreP) {
#pragma unroll
            for (int r = 0; r < R; ++r) pin[0][r] = X.pre[r];
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[j * R + r] = ptmul(conjg(v[j * R + r]), pin[j][r]);
        }
    } else if constexpr (MID == 2 || MID == 3 || MID == 9 || MID == 10) {
        // passes without a table: exp(-i phase v) in FP64 on the fly.  MID 3: the angle
        // phase v[n] + phase2 v2[n] of a time-dependent potential, both fields in FP64
        if constexpr (MID == 9 || MID == 10) {
            if (a.sum_part) tile_sums<T, E, NT, J, R, false>(a, tile, b, v, voff, rstep, nullptr);
        }
        double pin[J][R];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int bf = threadIdx.x + j * NT;
            const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t n = (int64_t)(t + r * BPS) * L2 + c0 + q;
                pin[j][r] = n < a.Nvalid ? a.v[b * a.v_bs + n] : 0.0;
            }
        }
        if constexpr (MID == 3) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int bf = threadIdx.x + j * NT;
                const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t n = (int64_t)(t + r * BPS) * L2 + c0 + q;
                    pin[j][r] = a.phase * pin[j][r] + (n < a.Nvalid ? a.phase2 * a.v2[b * a.v_bs + n] : 0.0);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int bf = threadIdx.x + j * NT;
            const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t n = (int64_t)(t + r * BPS) * L2 + c0 + q;
                const double ang = MID == 3 ? pin[j][r] : a.phase * pin[j][r];
                // MID 9 holds the input's point values, the others the
                // conjugates left by the inverse DFT
                const cx<T> x = MID == 9 ? v[j * R + r] : conjg(v[j * R + r]);
                v[j * R + r] = n < a.Nvalid ? mul_expm_i(x, ang) : cx<T>{0, 0};
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        int pin[J][R];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int bf = threadIdx.x + j * NT;
            const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t n = (int64_t)(t + r * BPS) * L2 + c0 + q;
                pin[j][r] = n < a.Nvalid ? a.s[n] : -1;
            }
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int m = pin[j][r];
                v[j * R + r] = m >= 0 ? cmul_d(conjg(v[j * R + r]), a.ktab[2 * m], a.ktab[2 * m + 1]) : cx<T>{0, 0};
            }
        }
    }
    if constexpr (kFwd) F::run(v, s, B, kInv || sync_first);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (kFwd && tw) apply_series<T, R>(&v[j * R], tb[j], ts[j]);
#pragma unroll
        for (int r = 0; r < R; ++r) bstore<SA>(v[j * R + r], rb, voff[j], r * rstep);
    }
    (void)TILE;
}

// S column tiles per workgroup (consecutive tiles S w .. S w + S - 1): the
// loads of all S tiles are issued first, so that the later tiles' loads are
// in flight while the first tiles are transformed, and the first tiles'
// stores drain while the later ones are.
template <typename T, int E, int NT, int MID, int S, int SA, int... Rs>
__device__ __forceinline__ void colf_body(const ColArgs &a, int wtile, int64_t b, cx<T> *s)
{
    using F = Fft<T, E, NT, true, Rs...>;
    constexpr bool PRE = col_prefetch<T, MID, F::J, S>();
    constexpr bool PV = col_prefetch_v<MID, E>();
    typename F::Bases B;
    F::load_bases(B, (const Tw<T> *)a.twa);
    ColTile<T, E, F::J, F::R, PRE, PV> X[S];
#pragma unroll
    for (int st = 0; st < S; ++st) colf_load<T, E, NT, PRE, PV, MID == 9, Rs...>(a, wtile * S + st, b, X[st]);
#pragma unroll
    for (int st = 0; st < S; ++st)
        colf_run<T, E, NT, MID, PRE, PV, SA, Rs...>(a, wtile * S + st, b, s, B, X[st], st > 0);
}

template <typename T, int E, int NT, int MINW, int MID, int SA, int... Rs>
__global__ void __launch_bounds__(NT, MINW) k_colf(ColArgs a)
{
    extern __shared__ char smem_raw[];
    colf_body<T, E, NT, MID, 1, SA, Rs...>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.y,
                                           reinterpret_cast<cx<T> *>(smem_raw));
}

// two column tiles per workgroup
template <typename T, int E, int NT, int MINW, int MID, int SA, int... Rs>
__global__ void __launch_bounds__(NT, MINW) k_colf2(ColArgs a)
{
    extern __shared__ char smem_raw[];
    colf_body<T, E, NT, MID, 2, SA, Rs...>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.y,
                                           reinterpret_cast<cx<T> *>(smem_raw));
}

// Interior merge pass of the adjoint sweep (no checkpoint reset, no chirp):
// the tile holds C/2 state columns (sequences q < C/2, buffer buf) and the
// same C/2 cotangent columns (sequences q >= C/2, buffer buf2, which follows
// buf in the same allocation).  After the inverse column DFTs the two values
// of each point meet through LDS: a = state, mu = cotangent;
// dJ/dv[n] += gcoef Im(conj(mu) a); both are multiplied by exp(-i phase v[n])
// from the sweep's table; then the forward column DFTs.  Both vectors are
// addressed through one buffer resource (the cotangent at a fixed element
// offset), and every accumulator and table entry a thread touches is loaded
// before the first use.
template <typename T, int E, int NT, int MINW, int... Rs>
__global__ void __launch_bounds__(NT, MINW) k_colf_adj(ColArgs a)
{
    using F = Fft<T, E, NT, true, Rs...>;
    constexpr int C = F::SEQ, H = C / 2, J = F::J, R = F::R, BPS = F::BPS, L1 = F::L;
    static_assert(C % 2 == 0, "state and cotangent columns pair up");
    constexpr int IT = H * L1 / NT;  // points per thread in the pairing step
    static_assert((H * L1) % NT == 0, "whole pairing iterations");
    extern __shared__ char smem_raw[];
    cx<T> *s = reinterpret_cast<cx<T> *>(smem_raw);
    const int L2 = a.L2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t b = blockIdx.y;
    const int c0 = tile * H;
    cx<T> *base = (cx<T> *)a.buf + b * a.buf_bs;
    const uint32_t delta = (uint32_t)((cx<T> *)a.buf2 - (cx<T> *)a.buf);  // cotangent offset, elements
    const rsrc_t rb = make_rsrc(base, ((int64_t)delta + (int64_t)L1 * L2) * (int64_t)sizeof(cx<T>));
    constexpr uint32_t S = (uint32_t)sizeof(cx<T>);
    const uint32_t rstep = (uint32_t)BPS * (uint32_t)L2 * S;
    typename F::Bases B;
    F::load_bases(B, (const Tw<T> *)a.twa);
    uint32_t voff[J];
    cx<T> v[E];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int bf = threadIdx.x + j * NT;
        const int q = F::q_of(bf), t = F::t_of(bf);
        const uint32_t n2 = (uint32_t)(c0 + (q < H ? q : q - H));
        voff[j] = ((uint32_t)t * (uint32_t)L2 + n2 + (q < H ? 0u : delta)) * S;
#pragma unroll
        for (int r = 0; r < R; ++r) v[j * R + r] = bload<T>(rb, voff[j], r * rstep);
    }
    const bool tw = a.twiddle != 0;
    cx<double> tb[J], ts[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        tb[j] = {1.0, 0.0};
        ts[j] = {1.0, 0.0};
    }
    if (tw) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int bf = threadIdx.x + j * NT;
            const int q = F::q_of(bf);
            tw4_base_step(tb[j], ts[j], c0 + (q < H ? q : q - H), F::t_of(bf), BPS, L2, a.tw4hi, a.tw4lo);
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[j * R + r] = conjg(v[j * R + r]);
        if (tw) apply_series<T, R>(&v[j * R], tb[j], ts[j]);
    }
    F::run(v, s, B, false);
    // pair the two vectors of each point through LDS
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int bf = threadIdx.x + j * NT;
        const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
        for (int r = 0; r < R; ++r) s[F::addr(q, t + r * BPS)] = conjg(v[j * R + r]);
    }
    // the accumulator and table entries of this thread's points, all in flight
    // at once (point n = k1 L2 + c0 + q of iteration it; the buffers' range
    // checks read the zero padding n >= Nvalid as 0 and drop its stores)
    const rsrc_t rg = make_rsrc(a.gacc + b * a.gacc_bs, a.Nvalid * (int64_t)sizeof(double));
    const rsrc_t rp = make_rsrc((const PTab<T> *)a.ptab + b * a.ptab_bs, a.Nvalid * (int64_t)sizeof(PTab<T>));
    double g_in[IT];
    PTab<T> pw[IT];
    uint32_t nn[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * NT;
        const int k1 = i / H, q = i - k1 * H;
        nn[it] = (uint32_t)k1 * (uint32_t)L2 + (uint32_t)(c0 + q);
        g_in[it] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rg, nn[it] * 8u, 0, 0));
        pw[it] = pload<T>(rp, nn[it] * (uint32_t)sizeof(PTab<T>));
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * NT;
        const int k1 = i / H, q = i - k1 * H;
        const int ax = F::addr(q, k1), ay = F::addr(q + H, k1);
        if ((int64_t)nn[it] >= a.Nvalid) {
            s[ax] = {0, 0};
            s[ay] = {0, 0};
            continue;
        }
        const cx<T> x = s[ax], y = s[ay];
        const double im = (double)y.x * (double)x.y - (double)y.y * (double)x.x;
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(rg, 0, 0, 0)), g_in[it] + a.gcoef * im),
            rg, nn[it] * 8u, 0, 0);
        const cx<double> w = pt_d(pw[it]);  // the sweep's table of exp(-i phase v[n])
        s[ax] = cmul_d(x, w.x, w.y);
        s[ay] = cmul_d(y, w.x, w.y);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int bf = threadIdx.x + j * NT;
        const int q = F::q_of(bf), t = F::t_of(bf);
#pragma unroll
        for (int r = 0; r < R; ++r) v[j * R + r] = s[F::addr(q, t + r * BPS)];
    }
    F::run(v, s, B, true);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (tw) apply_series<T, R>(&v[j * R], tb[j], ts[j]);
#pragma unroll
        for (int r = 0; r < R; ++r) bstore(v[j * R + r], rb, voff[j], r * rstep);
    }
}

// Pass g of the batch members listed in idx (prefix sums of their column
// tiles in start, block offset off).  MID 0: the merged potential step of
// each member whose schedule is at an interior column pass; MID 9: the
// members' first pass (g = 0); MID 10: the last pass of each member whose
// schedule ends at g.  The members' tiles are counted in 4096-element tiles;
// a kernel with Q times smaller tiles runs Q blocks per counted tile.
template <typename T, int E, int NT, int MINW, int MID, int Q, int... Rs>
__global__ void __launch_bounds__(NT, MINW) k_colf_multi(const BatchDesc *d, const int *idx, const int *start,
                                                          int nmem, int nblocks, int off, int64_t g)
{
    extern __shared__ char smem_raw[];
    // the grid is padded to a multiple of 8 blocks
    const int w = xcd_block(blockIdx.x, gridDim.x);
    if (w >= nblocks * Q) return;
    const int bid = w / Q + off;
    const int k = find_member(start, nmem, bid);
    const BatchDesc &p = d[idx[k]];
    if constexpr (MID == 9) {
        if (g != 0) return;
    } else if constexpr (MID == 10) {
        if (g != p.npass - 1) return;
    } else {
        if (g == 0 || (g & 1) || g >= p.npass - 1) return;
    }
    // members with interior passes carry the per-point table of the merged
    // potential step (col[1]); col[0] and col[3] are the first and last roles
    colf_body<T, E, NT, MID, 1, 0, Rs...>(p.col[MID == 9 ? 0 : MID == 10 ? 3 : 1], (bid - start[k]) * Q + w % Q, 0,
                                       reinterpret_cast<cx<T> *>(smem_raw));
}

// Row pass: [DFT -> spectral multiplier -> inverse DFT], in place; the
// multiplier (chirp-z kernel spectrum or kinetic table) is applied in registers.
template <typename T, int E, int NT, int MID, int SA, int... Rs>
__device__ __forceinline__ void rowf_body(const RowArgs &a, int blk, int64_t b, cx<T> *s)
{
    using F = Fft<T, E, NT, false, Rs...>;
    constexpr int L2 = F::L, RW = F::SEQ, J = F::J, R = F::R, BPS = F::BPS, TILE = F::TILE;
    const int r0 = blk * RW;
    cx<T> *buf = (cx<T> *)a.buf + b * a.buf_bs + (int64_t)r0 * L2;
    typename F::Bases B;
    F::load_bases(B, (const Tw<T> *)a.twb);
    const int64_t p0 = (int64_t)r0 * L2;
    // element (q, t + r BPS) of the block sits at byte voff[j] + r * rstep
    const rsrc_t rb = make_rsrc(buf, (int64_t)TILE * (int64_t)sizeof(cx<T>));
    constexpr uint32_t rstep = (uint32_t)BPS * (uint32_t)sizeof(cx<T>);
    uint32_t voff[J];
    cx<T> v[E];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int bf = threadIdx.x + j * NT;
        voff[j] = (uint32_t)(F::q_of(bf) * L2 + F::t_of(bf)) * (uint32_t)sizeof(cx<T>);
#pragma unroll
        for (int r = 0; r < R; ++r) v[j * R + r] = bload<T>(rb, voff[j], r * rstep);
    }
    // kinetic table: the squared-norm index of every element (4 bytes at the
    // element's offset scaled by 4 / sizeof(cx<T>)); after the forward DFT
    // each thread holds the spectrum at the same positions, so the
    // multiplier is applied in registers.  The indices are loaded with the
    // state, except in the complex128 8192-point rows, where holding them
    // through the DFT would spill.
    constexpr bool kPreS = MID == 1 && !(sizeof(T) == 8 && TILE > 4096);
    int sk[MID == 1 ? E : 1];
    auto load_sk = [&]() {
        const rsrc_t rs = make_rsrc(a.s + p0, (int64_t)TILE * 4);
        constexpr uint32_t ss = (uint32_t)sizeof(cx<T>) / 4;
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                sk[j * R + r] = (int)__builtin_amdgcn_raw_buffer_load_b32(rs, voff[j] / ss, r * (rstep / ss), 0);
        }
    };
    if constexpr (kPreS) load_sk();
    F::run(v, s, B, false);
    if constexpr (MID == 1 && !kPreS) load_sk();
    if constexpr (MID == 0) {
        // chirp-z kernel spectrum: one complex-double load per element, at the
        // element's offset scaled by 16 / sizeof(cx<T>)
        const rsrc_t rg = make_rsrc(a.bhat + 2 * p0, (int64_t)TILE * 16);
        constexpr uint32_t gs = 16 / (uint32_t)sizeof(cx<T>);
        cx<double> g[E];
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) g[j * R + r] = bload<double>(rg, gs * voff[j], gs * r * rstep);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const cx<double> w = g[j * R + r];
                v[j * R + r] = conjg(cmul_d(v[j * R + r], w.x, a.conj_tab ? -w.y : w.y));
            }
        }
    } else if constexpr (MID == 2) {
        // complex64: the spectrum rounded once to complex float, 8 bytes per
        // element at the element's own offset, applied in float
        static_assert(sizeof(T) == 4, "complex-float spectrum rows are complex64 only");
        const rsrc_t rg = make_rsrc(a.bhat_f + 2 * p0, (int64_t)TILE * 8);
        cx<float> g[E];
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int r = 0; r < R; ++r) g[j * R + r] = bload<float>(rg, voff[j], r * rstep);
        }
        const float sg = a.conj_tab ? -1.0f : 1.0f;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cx<T> x = v[e];
            const float gx = g[e].x, gy = sg * g[e].y;
            v[e] = conjg(cx<T>{x.x * gx - x.y * gy, x.x * gy + x.y * gx});
        }
    } else {
        // kinetic table indexed by the squared norm (a small table, cached):
        // every entry of the thread in flight at once
        const rsrc_t rk = make_rsrc(a.ktab, a.ktab_n * 16);
        constexpr int KC = kPreS ? E : 8;  // entries in flight (fewer where registers are short)
#pragma unroll
        for (int e0 = 0; e0 < E; e0 += KC) {
            cx<double> k[KC];
#pragma unroll
            for (int e = 0; e < KC; ++e) k[e] = bload<double>(rk, (uint32_t)sk[e0 + e] * 16u, 0);
#pragma unroll
            for (int e = 0; e < KC; ++e) v[e0 + e] = conjg(cmul_d(v[e0 + e], k[e].x, k[e].y));
        }
    }
    F::run(v, s, B, true);
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
        for (int r = 0; r < R; ++r) bstore<SA>(conjg(v[j * R + r]), rb, voff[j], r * rstep);
    }
}

template <typename T, int E, int NT, int MINW, int MID, int SA, int... Rs>
__global__ void __launch_bounds__(NT, MINW) k_rowf(RowArgs a)
{
    extern __shared__ char smem_raw[];
    rowf_body<T, E, NT, MID, SA, Rs...>(a, blockIdx.x, blockIdx.y, reinterpret_cast<cx<T> *>(smem_raw));
}

// Row pass g of the batch members listed in idx (prefix sums of their row
// blocks in start, block offset off); MID 0: spectrum table, MID 1: kinetic
// table, MID 2: spectrum in complex float, as in k_rowf.  Q blocks per counted 4096-element block, as in
// k_colf_multi.
template <typename T, int E, int NT, int MINW, int MID, int Q, int... Rs>
__global__ void __launch_bounds__(NT, MINW) k_rowf_multi(const BatchDesc *d, const int *idx, const int *start,
                                                          int nmem, int nblocks, int off, int64_t g)
{
    extern __shared__ char smem_raw[];
    if ((int)blockIdx.x >= nblocks * Q) return;
    const int bid = (int)blockIdx.x / Q + off;
    const int k = find_member(start, nmem, bid);
    const BatchDesc &p = d[idx[k]];
    if (!(g & 1) || g >= p.npass) return;
    rowf_body<T, E, NT, MID, 0, Rs...>(p.row[0], (bid - start[k]) * Q + (int)blockIdx.x % Q, 0,
                                    reinterpret_cast<cx<T> *>(smem_raw));
}

// ---------------------------------------------------------------- dispatch
// Variant 1: 256 threads x 16 elements (radix 16 / 8); variant 2: 512 threads
// x 8 elements (radix 8 / 4, twice the waves per CU).  Both hold a
// 4096-element tile, so they share the plan's layout and are interchangeable.
namespace {
constexpr int kTile = 4096;  // elements of the tile a plan counts its column and row tiles in

template <int V>
struct Geo;
template <>
struct Geo<1> {
    static constexpr int NT = 256, E = 16, MINW = 2;
};
template <>
struct Geo<2> {
    static constexpr int NT = 512, E = 8, MINW = 4;
};
template <>
struct Geo<3> {  // rows of kWideRow points: one row per workgroup
    static constexpr int NT = 512, E = 16, MINW = 1;
};
template <>
struct Geo<4> {  // small tiles (one wave, 1024 elements): more workgroups for small transforms
    static constexpr int NT = 64, E = 16, MINW = 2;
};
template <>
struct Geo<5> {  // 512 threads x 8 with the register budget of two waves per SIMD: two
                 // 4096-element column tiles per workgroup, or one row tile
    static constexpr int NT = 512, E = 8, MINW = 2, S = 2;
};
template <>
struct Geo<6> {  // 256 threads x 8 (2048-element tiles): twice the workgroups of
                 // 1, 2 and 4 at two waves per SIMD, for transforms of 2^20 points
    static constexpr int NT = 256, E = 8, MINW = 2;
};
template <int V>
constexpr int tiles_per_group()
{
    if constexpr (V == 5) return Geo<5>::S;
    else return 1;
}

// the column kernel for S tiles per workgroup and store policy SA
template <typename T, int E, int NT, int MINW, int MID, int S, int SA, int... Rs>
constexpr auto colk()
{
    if constexpr (S == 2) return k_colf2<T, E, NT, MINW, MID, SA, Rs...>;
    else return k_colf<T, E, NT, MINW, MID, SA, Rs...>;
}

template <typename K, typename A>
int timed(int kind, K kernel, dim3 grid, dim3 block, size_t lds, void *stream, const A &args)
{
    void *e0 = nullptr, *e1 = nullptr;
    timing_events(kind, &e0, &e1);
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, block, lds, (hipStream_t)stream, (hipEvent_t)e0, (hipEvent_t)e1, 0,
                              args);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, (hipStream_t)stream, args);
    return (int)hipGetLastError();
}

template <typename K, typename... A>
int timed_multi(int kind, K kernel, dim3 grid, dim3 block, size_t lds, void *stream, A... args)
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

template <typename T, int V>
size_t lds_bytes()
{
    constexpr int tile = Geo<V>::NT * Geo<V>::E;
    return (size_t)(tile + tile / 16) * sizeof(cx<T>);
}

template <typename T, int V, int... Rs>
int col_go(const ColArgs &a, int batch, void *stream)
{
    constexpr int NT = Geo<V>::NT, E = Geo<V>::E, MINW = Geo<V>::MINW, S = tiles_per_group<V>();
    // MID 0: merged potential step from the per-point table; MID 1: kinetic table;
    // MID 2 (complex128 runs without a table): FP64 phase of v; MID 3:
    // potential with a time-dependent second field
    auto k = colk<T, E, NT, MINW, 1, S, 0, Rs...>();
    if (a.pre_inv != a.post_fwd && a.v) {
        // a run's first (forward only) or last (inverse only) pass: the half
        // potential step from v in FP64, and the step's sums when asked for
        if (a.v2 || a.ptab || a.ktab || a.ck || a.chirp || (a.sum_part && !a.sum_v)) return -1;
        k = a.post_fwd ? colk<T, E, NT, MINW, 9, S, 0, Rs...>() : colk<T, E, NT, MINW, 10, S, 0, Rs...>();
        static bool attr_end = false;
        if (!attr_end) {
            hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 9, S, 0, Rs...>(),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
            hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 10, S, 0, Rs...>(),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
            attr_end = true;
        }
        constexpr int C = NT * E / Radix<Rs...>::prod;
        if (a.L2 % (C * S)) return -1;
        return timed(LT_KIND_COLUMN, k, dim3(a.L2 / (C * S), batch), dim3(NT), lds_bytes<T, V>(), stream, a);
    }
    if constexpr (V == 1) {
        if (a.pre_inv != a.post_fwd) {
            k = a.post_fwd ? k_colf<T, E, NT, MINW, 5, 0, Rs...> : k_colf<T, E, NT, MINW, 6, 0, Rs...>;
            static bool attr_io = false;
            if (!attr_io) {
                hipFuncSetAttribute((const void *)k_colf<T, E, NT, MINW, 5, 0, Rs...>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
                hipFuncSetAttribute((const void *)k_colf<T, E, NT, MINW, 6, 0, Rs...>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
                attr_io = true;
            }
            constexpr int C = NT * E / Radix<Rs...>::prod;
            return timed(LT_KIND_COLUMN, k, dim3(a.L2 / C, batch), dim3(NT), lds_bytes<T, V>(), stream, a);
        }
    } else {
        if (a.pre_inv != a.post_fwd) return -1;
    }
    if (a.ck) {  // checkpoint pass (and the step's sums, when asked for)
        if (!a.v || a.v2 || !a.ptab) return -1;
        k = colk<T, E, NT, MINW, 7, S, 0, Rs...>();
    } else if (a.sum_part) {  // merged step plus the step's sums in registers
        if (!a.v || a.v2 || !a.ptab || !a.sum_v) return -1;
        k = a.wt ? colk<T, E, NT, MINW, 8, S, kWriteThrough, Rs...>() : colk<T, E, NT, MINW, 8, S, 0, Rs...>();
    } else if (a.v) {
        if (a.v2) k = colk<T, E, NT, MINW, 3, S, 0, Rs...>();
        else if (a.ptab)
            k = a.wt ? colk<T, E, NT, MINW, 0, S, kWriteThrough, Rs...>() : colk<T, E, NT, MINW, 0, S, 0, Rs...>();
        else if constexpr (sizeof(T) == 8) k = colk<T, E, NT, MINW, 2, S, 0, Rs...>();
        else return -1;
    }
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 0, S, 0, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 1, S, 0, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 3, S, 0, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 7, S, 0, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 8, S, 0, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        if constexpr (sizeof(T) == 8)
            hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 2, S, 0, Rs...>(),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 0, S, kWriteThrough, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)colk<T, E, NT, MINW, 8, S, kWriteThrough, Rs...>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        attr = true;
    }
    constexpr int C = NT * E / Radix<Rs...>::prod;
    if (a.L2 % (C * S)) return -1;
    dim3 grid(a.L2 / (C * S), batch);
    const size_t lds = lds_bytes<T, V>();
    return timed(LT_KIND_COLUMN, k, grid, dim3(NT), lds, stream, a);
}

template <typename T, int V, int... Rs>
int row_go(const RowArgs &a, int batch, void *stream)
{
    constexpr int NT = Geo<V>::NT, E = Geo<V>::E, MINW = Geo<V>::MINW;
    auto k = a.bhat ? k_rowf<T, E, NT, MINW, 0, 0, Rs...> : k_rowf<T, E, NT, MINW, 1, 0, Rs...>;
    if (a.wt)
        k = a.bhat ? k_rowf<T, E, NT, MINW, 0, kWriteThrough, Rs...> : k_rowf<T, E, NT, MINW, 1, kWriteThrough, Rs...>;
    if constexpr (sizeof(T) == 4) {
        // complex64 with the spectrum in complex float
        if (a.bhat_f) k = a.wt ? k_rowf<T, E, NT, MINW, 2, kWriteThrough, Rs...> : k_rowf<T, E, NT, MINW, 2, 0, Rs...>;
        static bool attr_f = false;
        if (!attr_f) {
            hipFuncSetAttribute((const void *)k_rowf<T, E, NT, MINW, 2, 0, Rs...>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
            hipFuncSetAttribute((const void *)k_rowf<T, E, NT, MINW, 2, kWriteThrough, Rs...>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
            attr_f = true;
        }
    }
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void *)k_rowf<T, E, NT, MINW, 0, 0, Rs...>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)k_rowf<T, E, NT, MINW, 1, 0, Rs...>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)k_rowf<T, E, NT, MINW, 0, kWriteThrough, Rs...>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        hipFuncSetAttribute((const void *)k_rowf<T, E, NT, MINW, 1, kWriteThrough, Rs...>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        attr = true;
    }
    constexpr int RW = NT * E / Radix<Rs...>::prod;
    dim3 grid(a.L1 / RW, batch);
    const size_t lds = lds_bytes<T, V>();
    return timed(LT_KIND_ROW, k, grid, dim3(NT), lds, stream, a);
}

template <typename T, int V, bool COL, int... Rs, class A>
int go1(const A &a, int batch, void *stream)
{
    if constexpr (COL) return col_go<T, V, Rs...>(a, batch, stream);
    else return row_go<T, V, Rs...>(a, batch, stream);
}

// radix sequence of each supported length per variant (first radix = last;
// every radix divides the elements per thread)
template <typename T, int V, bool COL, class A>
int go(int L, const A &a, int batch, void *stream)
{
    if constexpr (V == 3) {  // 16 elements per thread, 512 threads: rows of 8192, pairs of 4096-point columns
        if (L == 8192 && !COL) return go1<T, V, COL, 16, 4, 8, 16>(a, batch, stream);
        if (L == 4096 && COL) return go1<T, V, COL, 16, 16, 16>(a, batch, stream);
        return -1;
    } else if constexpr (V == 4) {  // 16 elements per thread, 64 threads: lengths up to 1024
        switch (L) {
        case 64: return go1<T, V, COL, 8, 8>(a, batch, stream);
        case 128: return go1<T, V, COL, 8, 2, 8>(a, batch, stream);
        case 256: return go1<T, V, COL, 16, 16>(a, batch, stream);
        case 512: return go1<T, V, COL, 8, 8, 8>(a, batch, stream);
        case 1024: return go1<T, V, COL, 16, 4, 16>(a, batch, stream);
        default: return -1;
        }
    } else if constexpr (V == 1) {  // 16 elements per thread
        switch (L) {
        case 64: return go1<T, V, COL, 8, 8>(a, batch, stream);
        case 128: return go1<T, V, COL, 8, 2, 8>(a, batch, stream);
        case 256: return go1<T, V, COL, 16, 16>(a, batch, stream);
        case 512: return go1<T, V, COL, 8, 8, 8>(a, batch, stream);
        case 1024: return go1<T, V, COL, 16, 4, 16>(a, batch, stream);
        case 2048: return go1<T, V, COL, 16, 8, 16>(a, batch, stream);
        case 4096: return go1<T, V, COL, 16, 16, 16>(a, batch, stream);
        default: return -1;
        }
    } else {  // 8 elements per thread
        switch (L) {
        case 64: return go1<T, V, COL, 8, 8>(a, batch, stream);
        case 128: return go1<T, V, COL, 8, 2, 8>(a, batch, stream);
        case 256: return go1<T, V, COL, 8, 4, 8>(a, batch, stream);
        case 512: return go1<T, V, COL, 8, 8, 8>(a, batch, stream);
        case 1024: return go1<T, V, COL, 8, 4, 4, 8>(a, batch, stream);
        case 2048: return go1<T, V, COL, 8, 4, 8, 8>(a, batch, stream);
        case 4096:
            if constexpr (V != 6) return go1<T, V, COL, 8, 8, 8, 8>(a, batch, stream);
            else return -1;  // longer than the 2048-element tile
        default: return -1;
        }
    }
}

bool fast_len(int L) { return L >= 64 && L <= 4096 && (L & (L - 1)) == 0; }

template <typename T, int V, int MID, int... Rs>
int col_multi_go(const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks, int off, int64_t g,
                 void *stream)
{
    constexpr int NT = Geo<V>::NT, E = Geo<V>::E, MINW = Geo<V>::MINW, Q = kTile / (NT * E);
    auto k = k_colf_multi<T, E, NT, MINW, MID, Q, Rs...>;
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        attr = true;
    }
    const int grid = (nblocks * Q + 7) / 8 * 8;
    return timed_multi(LT_KIND_COLUMN, k, dim3(grid), dim3(NT), lds_bytes<T, V>(), stream, d, idx, start, nmem,
                       nblocks, off, g);
}

template <typename T, int V, int MID, int... Rs>
int row_multi_go(const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks, int off, int64_t g,
                 void *stream)
{
    constexpr int NT = Geo<V>::NT, E = Geo<V>::E, MINW = Geo<V>::MINW, Q = kTile / (NT * E);
    auto k = k_rowf_multi<T, E, NT, MINW, MID, Q, Rs...>;
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        attr = true;
    }
    return timed_multi(LT_KIND_ROW, k, dim3(nblocks * Q), dim3(NT), lds_bytes<T, V>(), stream, d, idx, start, nmem,
                       nblocks, off, g);
}

// one multi-member launch: the column or the row kernel of the pass kind MID
template <typename T, bool COL, int MID, int V, int... Rs>
int multi_one(const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks, int off, int64_t g,
              void *stream)
{
    if constexpr (COL) return col_multi_go<T, V, MID, Rs...>(d, idx, start, nmem, nblocks, off, g, stream);
    else return row_multi_go<T, V, MID, Rs...>(d, idx, start, nmem, nblocks, off, g, stream);
}

// radix sequences per length of the two 4096-element-tile geometries (as in
// go<T, 1 or 2, ...>): variant 1 (256 threads x 16) and 2 (512 threads x 8)
template <typename T, bool COL, int MID, int V>
int multi_go_v(int L, const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks, int off,
               int64_t g, void *stream)
{
#define LT_MULTI(...) multi_one<T, COL, MID, V, __VA_ARGS__>(d, idx, start, nmem, nblocks, off, g, stream)
    if constexpr (V == 1) {
        switch (L) {
        case 64: return LT_MULTI(8, 8);
        case 128: return LT_MULTI(8, 2, 8);
        case 256: return LT_MULTI(16, 16);
        case 512: return LT_MULTI(8, 8, 8);
        case 1024: return LT_MULTI(16, 4, 16);
        case 2048: return LT_MULTI(16, 8, 16);
        case 4096: return LT_MULTI(16, 16, 16);
        default: return -1;
        }
    } else {
        switch (L) {
        case 64: return LT_MULTI(8, 8);
        case 128: return LT_MULTI(8, 2, 8);
        case 256: return LT_MULTI(8, 4, 8);
        case 512: return LT_MULTI(8, 8, 8);
        case 1024: return LT_MULTI(8, 4, 4, 8);
        case 2048: return LT_MULTI(8, 4, 8, 8);
        case 4096:
            if constexpr (V != 6) return LT_MULTI(8, 8, 8, 8);
            else return -1;  // longer than the 2048-element tile
        default: return -1;
        }
    }
#undef LT_MULTI
}

template <typename T, bool COL, int MID>
int multi_go(int variant, int L, const BatchDesc *d, const int *idx, const int *start, int nmem, int nblocks,
             int off, int64_t g, void *stream)
{
    if (variant == 2) return multi_go_v<T, COL, MID, 2>(L, d, idx, start, nmem, nblocks, off, g, stream);
    if (variant == 5) return multi_go_v<T, COL, MID, 6>(L, d, idx, start, nmem, nblocks, off, g, stream);
    return multi_go_v<T, COL, MID, 1>(L, d, idx, start, nmem, nblocks, off, g, stream);
}
}  // namespace

constexpr int kSmallTile = Geo<4>::NT * Geo<4>::E;

// variants 1 and 2 take the plan's tile (C columns / rows of a 4096-element
// tile); variant 3 uses its own tiles: 1024 elements for lengths up to 1024,
// and two 4096-point columns per 8192-element tile
bool fast_col_fits(int prec, int variant, int L1, int L2, int C)
{
    (void)prec;
    if (variant == 3)
        return (fast_len(L1) && L1 <= kSmallTile && L2 % (kSmallTile / L1) == 0) || (L1 == 4096 && L2 % 2 == 0);
    if (variant == 4) return fast_len(L1) && C == kTile / L1 && L2 % (2 * C) == 0;
    if (variant == 5) return fast_len(L1) && L1 <= kTile / 2 && L2 % (kTile / 2 / L1) == 0;
    return (variant == 1 || variant == 2) && fast_len(L1) && C == kTile / L1 && L2 % C == 0;
}

bool fast_row_fits(int prec, int variant, int L1, int L2, int rows)
{
    (void)prec;
    // rows of kWideRow points: one per workgroup, the 512-thread kernel (variants 1 and 2)
    if (L2 == kWideRow) return rows == 1 && (variant == 1 || variant == 2 || variant == 4);
    if (variant == 3) return fast_len(L2) && L2 <= kSmallTile && L1 % (kSmallTile / L2) == 0;
    if (variant == 5) return fast_len(L2) && L2 <= kTile / 2 && L1 % (kTile / 2 / L2) == 0;
    return (variant == 1 || variant == 2 || variant == 4) && fast_len(L2) && rows == kTile / L2 && L1 % rows == 0;
}

int launch_col_fast(int prec, int variant, const ColArgs &a, int batch, void *stream)
{
    // steady-state passes, and the first and last passes of runs without the
    // chirp-z pair form (the first reads the input vector, the last writes
    // the output vector); the adjoint passes and the general first / last
    // passes (chirp-z pair, scaled, time-dependent) take the general kernel
    const bool steady = a.pre_inv && a.post_fwd && !a.in && !a.out && !a.chirp && a.scale == 1.0 &&
                        !a.adjoint && ((a.v != nullptr) != (a.ktab != nullptr)) &&
                        (prec == LT_C128 || !a.v || a.ptab || a.v2) &&
                        (!a.ck || (a.ptab && a.v && !a.v2 && !a.ck_chirp && a.ck_v)) &&
                        (!a.sum_part || (a.ptab && a.v && !a.v2 && a.sum_v));
    const bool first = !a.pre_inv && a.post_fwd && a.in && !a.out;
    const bool last = a.pre_inv && !a.post_fwd && !a.in && a.out;
    const bool ends = (first || last) && a.v && !a.v2 && !a.ptab && !a.ktab && !a.ck && !a.chirp &&
                      a.scale == 1.0 && !a.adjoint && (!a.sum_part || a.sum_v);
    if (!(steady || ends) || !fast_col_fits(prec, variant, a.L1, a.L2, a.C)) return -1;
    if (variant == 3 && a.L1 == 4096)
        return prec == LT_C128 ? go<double, 3, true>(a.L1, a, batch, stream) : go<float, 3, true>(a.L1, a, batch, stream);
    if (prec == LT_C128)
        return variant == 1   ? go<double, 1, true>(a.L1, a, batch, stream)
               : variant == 2 ? go<double, 2, true>(a.L1, a, batch, stream)
               : variant == 4 ? go<double, 5, true>(a.L1, a, batch, stream)
               : variant == 5 ? go<double, 6, true>(a.L1, a, batch, stream)
                              : go<double, 4, true>(a.L1, a, batch, stream);
    return variant == 1   ? go<float, 1, true>(a.L1, a, batch, stream)
           : variant == 2 ? go<float, 2, true>(a.L1, a, batch, stream)
           : variant == 4 ? go<float, 5, true>(a.L1, a, batch, stream)
           : variant == 5 ? go<float, 6, true>(a.L1, a, batch, stream)
                          : go<float, 4, true>(a.L1, a, batch, stream);
}

int launch_col_inner(int prec, const ColArgs &a, int batch, void *stream)
{
    // a forward-only (post_fwd) or inverse-only (pre_inv) column pass in place,
    // the inner level of a three-level transform: register-staged kernel only
    const bool io = (a.pre_inv != a.post_fwd) && !a.in && !a.out && !a.v && !a.ktab && !a.ck && !a.chirp &&
                    a.scale == 1.0 && !a.adjoint;
    if (!io || !fast_col_fits(prec, 1, a.L1, a.L2, a.C)) return -1;
    return prec == LT_C128 ? go<double, 1, true>(a.L1, a, batch, stream) : go<float, 1, true>(a.L1, a, batch, stream);
}

int launch_row_fast(int prec, int variant, const RowArgs &a, int batch, void *stream)
{
    if (a.fft_only) return -1;
    if (a.L2 == kWideRow && a.rows == 1 && (variant == 1 || variant == 2 || variant == 4)) {
        if (prec == LT_C128) return go<double, 3, false>(a.L2, a, batch, stream);
        return go<float, 3, false>(a.L2, a, batch, stream);
    }
    if (!fast_row_fits(prec, variant, a.L1, a.L2, a.rows)) return -1;
    if (prec == LT_C128)
        return variant == 1   ? go<double, 1, false>(a.L2, a, batch, stream)
               : variant == 2 ? go<double, 2, false>(a.L2, a, batch, stream)
               : variant == 4 ? go<double, 5, false>(a.L2, a, batch, stream)
               : variant == 5 ? go<double, 6, false>(a.L2, a, batch, stream)
                              : go<double, 4, false>(a.L2, a, batch, stream);
    return variant == 1   ? go<float, 1, false>(a.L2, a, batch, stream)
           : variant == 2 ? go<float, 2, false>(a.L2, a, batch, stream)
           : variant == 4 ? go<float, 5, false>(a.L2, a, batch, stream)
           : variant == 5 ? go<float, 6, false>(a.L2, a, batch, stream)
                          : go<float, 4, false>(a.L2, a, batch, stream);
}

template <typename T, int... Rs>
int adj_go(const ColArgs &a, int batch, void *stream)
{
    constexpr int NT = Geo<1>::NT, E = Geo<1>::E, MINW = Geo<1>::MINW;
    auto k = k_colf_adj<T, E, NT, MINW, Rs...>;
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        attr = true;
    }
    constexpr int H = NT * E / Radix<Rs...>::prod / 2;
    return timed_multi(LT_KIND_COLUMN, k, dim3(a.L2 / H, batch), dim3(NT), lds_bytes<T, 1>(), stream, a);
}

template <typename T>
int adj_dispatch(const ColArgs &a, int batch, void *stream)
{
    switch (a.L1) {  // 4096-point columns leave one column per tile: no pairing
    case 64: return adj_go<T, 8, 8>(a, batch, stream);
    case 128: return adj_go<T, 8, 2, 8>(a, batch, stream);
    case 256: return adj_go<T, 16, 16>(a, batch, stream);
    case 512: return adj_go<T, 8, 8, 8>(a, batch, stream);
    case 1024: return adj_go<T, 16, 4, 16>(a, batch, stream);
    case 2048: return adj_go<T, 16, 8, 16>(a, batch, stream);
    default: return -1;
    }
}

int launch_col_fast_adjoint(int prec, int variant, const ColArgs &a, int batch, void *stream)
{
    if (variant < 1 || a.adjoint != 2 || a.reset || a.chirp || !a.pre_inv || !a.post_fwd || a.in || a.out ||
        !fast_len(a.L1) || a.L1 > 2048 || a.C != kTile / a.L1 / 2 || a.L2 % a.C || !a.ptab)
        return -1;
    // one buffer resource spans a state and its cotangent (which follows the
    // states in the same allocation): offsets stay below 2^31 bytes
    const int64_t S = prec == LT_C128 ? 16 : 8;
    if (a.buf2_bs != a.buf_bs) return -1;
    const int64_t delta = ((const char *)a.buf2 - (const char *)a.buf) / S;
    if (delta < 0 || (delta + (int64_t)batch * a.buf_bs + (int64_t)a.L1 * a.L2) * S >= (int64_t(1) << 31)) return -1;
    if (prec == LT_C128) return adj_dispatch<double>(a, batch, stream);
    return adj_dispatch<float>(a, batch, stream);
}

int launch_col_fast_multi(int prec, int variant, int L1, int mid, const BatchDesc *d, const int *idx,
                          const int *start, int nmem, int nblocks, int off, int64_t g, void *stream)
{
    // mid 0: interior passes, 9: first passes, 10: last passes
    if (mid != 0 && mid != 9 && mid != 10) return -1;
    if (prec == LT_C128) {
        if (mid == 9) return multi_go<double, true, 9>(variant, L1, d, idx, start, nmem, nblocks, off, g, stream);
        if (mid == 10) return multi_go<double, true, 10>(variant, L1, d, idx, start, nmem, nblocks, off, g, stream);
        return multi_go<double, true, 0>(variant, L1, d, idx, start, nmem, nblocks, off, g, stream);
    }
    if (mid == 9) return multi_go<float, true, 9>(variant, L1, d, idx, start, nmem, nblocks, off, g, stream);
    if (mid == 10) return multi_go<float, true, 10>(variant, L1, d, idx, start, nmem, nblocks, off, g, stream);
    return multi_go<float, true, 0>(variant, L1, d, idx, start, nmem, nblocks, off, g, stream);
}

int launch_row_fast_multi(int prec, int variant, int L2, int mid, const BatchDesc *d, const int *idx,
                          const int *start, int nmem, int nblocks, int off, int64_t g, void *stream)
{
    // mid 0: spectrum (complex double), 1: kinetic table, 2: spectrum in
    // complex float (complex64 only; every member's row carries bhat_f)
    if (prec == LT_C128) {
        if (mid == 2) return -1;
        return mid ? multi_go<double, false, 1>(variant, L2, d, idx, start, nmem, nblocks, off, g, stream)
                   : multi_go<double, false, 0>(variant, L2, d, idx, start, nmem, nblocks, off, g, stream);
    }
    if (mid == 2) return multi_go<float, false, 2>(variant, L2, d, idx, start, nmem, nblocks, off, g, stream);
    return mid ? multi_go<float, false, 1>(variant, L2, d, idx, start, nmem, nblocks, off, g, stream)
               : multi_go<float, false, 0>(variant, L2, d, idx, start, nmem, nblocks, off, g, stream);
}

}  // namespace lt
