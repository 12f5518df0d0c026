// Vertical-line block-Jacobi sweep (paper Eq. 1, Section 2.1) on the levels
// large enough to fill the GPU:
//   x_new = (1 - omega) x + omega H_z^{-1} (f + sum_h T_h x_nb)
// or, from zero, x_new = omega H_z^{-1} f.
//
// Each column's tridiagonal system is solved by the twisted factorisation of
// H_z: a pair of wavefronts takes a row-aligned segment of up to 64 columns,
// the bottom wavefront eliminates the layers below the meeting layer
// m = nz/2 going up, the top wavefront the layers above m going down, they
// meet at m through LDS, and each back-substitutes outward from registers.
//
// The kernel is written so that a step of the recurrence costs only its
// arithmetic:
//  - Every per-cell array of a level shares one layout, so one scalar byte
//    offset (layer * plane * sizeof(T)) addresses layer k in all of them;
//    loads and stores are buffer instructions with a per-lane column offset
//    and that shared scalar offset, with no per-lane address arithmetic.
//  - The row's couplings of step t (Tlam, Ttheta south and north, and the
//    vertical coupling to the next layer in the wavefront's direction) are
//    one 4-value record of a per-level table in step order, read with a
//    single scalar load whose offset is a compile-time constant.
//  - The layer loop is unrolled over a compile-time step count; on levels
//    whose layer count is the compiled one (EX), every role decision (which
//    steps eliminate, which one meets, which ones store) is a constant.
// Loads of the next chunk of D layers are issued before the current chunk
// is solved.
#include "device.hpp"

namespace mgk {

namespace {
using namespace dev;

// Per instantiation: D layers per prefetch chunk (5 divides the 35 steps of
// a 70-layer wavefront; 4 otherwise), W waves per SIMD (the register
// budget), KX: keep the old iterate of the half-column in LDS between the two
// passes (FP32 up to 72 layers; else it is loaded again, one chunk ahead,
// in the back-substitution). Measured on the 1024x768x70 shell: chunks of
// 7 layers, four waves per SIMD, one or four pairs per block, and a
// wavefront sweeping two or four segments in turn (the next segment's loads
// in flight during the back-substitution of the current one) were all
// within 2 % of this choice or slower.
template <typename T, int NZ, bool EX>
struct SweepCfg {
    static constexpr bool F32 = std::is_same<T, float>::value;
    static constexpr int NS0 = EX ? NZ - NZ / 2 : (NZ + 1) / 2;   // ceil(nz / 2)
    static constexpr bool SHORT = NS0 <= 36;
    static constexpr int D = F32 ? (EX && NS0 % 5 == 0 ? 5 : 4) : (EX ? 3 : 2);
    static constexpr int W = F32 && SHORT ? 3 : 2;
    static constexpr bool KX = F32 && EX && SHORT;
    static constexpr int NS = ((NS0 + D - 1) / D) * D;            // padded to whole chunks
};
// wavefront pairs per block
constexpr int kSweepPairs = 2;
constexpr bool kSweepShift = true;

// The raw loads of one step: right-hand side, inverse pivot, and the old
// iterate at the cell and its four horizontal neighbours.
template <typename T>
struct Raw {
    T f, ip, c, w, e, s, n;
};

// The column data of one wavefront's segment: per-lane byte offsets of the
// column and its four neighbours within a layer, validity, and its row's
// step records.
template <typename T>
struct SegData {
    uint32_t oc, ow, oe, os, on, og;
    bool valid;
    const StepCoef<T>* cr;
    __device__ __forceinline__ SegData(const LevelView<T>& L, int tile, int pair, bool top,
                                       int wpr) {
        const Seg g = tiled_segment(tile, pair, kSweepPairs, L.nI, L.nJ, wpr);
        oc = g.c * sizeof(T);
        ow = g.w * sizeof(T);
        oe = g.e * sizeof(T);
        og = (threadIdx.x & 63u) == 0 ? ow : oe;
        os = g.s * sizeof(T);
        on = g.n * sizeof(T);
        valid = g.valid;
        cr = L.sc + (size_t(top) * size_t(L.nJ) + size_t(g.J)) * kStepStride;
    }
};

// EX: nz == NZ. FULL: every lane of every wavefront has a column of its
// own (nI a multiple of 64, nJ of the pairs per block): no store is guarded.
// Cache policy CP by level: 0 plain loads and stores; 1 (levels of at
// least kSweepStreamCells cells) the new iterate stored with the
// non-temporal hint; 2 (fields of at least kStreamFieldBytes) the
// right-hand side and the pivots loaded with it as well. Smaller levels keep
// them in the caches for the next kernel.
constexpr long long kSweepStreamCells = 1LL << 23;

template <typename T, int NZ, bool EX, bool FULL, bool HAS_X, int CP>
__global__ __launch_bounds__(128 * kSweepPairs)
__attribute__((amdgpu_waves_per_eu(SweepCfg<T, NZ, EX>::W)))
void k_sweep(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ xin,
             T* __restrict__ xout, T omega, int wpr) {
    using C = SweepCfg<T, NZ, EX>;
    constexpr int D = C::D;
    constexpr int NS = C::NS;
    constexpr int NC = NS / D;
    constexpr bool KX = HAS_X && C::KX;
    // every lane has a column and loads the old iterate at it: the longitude
    // neighbours are the neighbour lanes' (lanes 0 and 63 load theirs)
    constexpr bool SHIFT = KX && FULL && kSweepShift;
    // the FP32 sweep from zero stores with plain stores even on large levels
    // (measured: 1-2% faster solves with it than with the hint)
    constexpr bool NT_STORE = CP >= 1 && (HAS_X || !std::is_same<T, float>::value);
    constexpr bool NT_LOAD = CP >= 2;
    static_assert(NS <= kStepStride, "step table too short");
    // the meeting exchange of each pair
    __shared__ T xch[kSweepPairs][4][64];

    const PairOf p = pair_of_wave();
    const bool top = p.top;
    const int lane = int(threadIdx.x & 63u);
    const int nz = EX ? NZ : L.nz;
    const int M = nz >> 1, TM = nz - 1 - M;    // meeting layer; top's elimination steps
    const uint32_t Pb = uint32_t(L.plane) * uint32_t(sizeof(T));
    const uint32_t bytes = Pb * uint32_t(nz);
    const rsrc_t rf = make_rsrc(f, bytes), rp = make_rsrc(L.invp, bytes),
                 rx = make_rsrc(HAS_X ? xin : f, bytes), ro = make_rsrc(xout, bytes);
    const T keep = T(1) - omega;

    // layer of step t, clamped (steps past a wavefront's layers load real
    // data and are discarded). Pbi is an opaque copy of the layer stride, so
    // that the compiler forms each offset where it is used instead of
    // keeping all of them in scalar registers.
    uint32_t Pbi = Pb;
    auto soff = [&](int t) -> uint32_t {
        int k = top ? nz - 1 - t : t;
        k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
        return uint32_t(k) * Pbi;
    };
    auto fetch = [&](const SegData<T>& sd, int t) {
        Raw<T> r;
        const uint32_t so = soff(t);
        r.f = bld<T, NT_LOAD>(rf, sd.oc, so);
        r.ip = bld<T, NT_LOAD>(rp, sd.oc, so);
        if constexpr (HAS_X) {
            if constexpr (SHIFT) {
                r.w = bld<T>(rx, sd.og, so);   // the segment's edges
            } else {
                r.w = bld<T>(rx, sd.ow, so);
                r.e = bld<T>(rx, sd.oe, so);
            }
            r.s = bld<T>(rx, sd.os, so);
            r.n = bld<T>(rx, sd.on, so);
            if constexpr (KX) r.c = bld<T>(rx, sd.oc, so);
        }
        return r;
    };
    auto comb = [&](const Raw<T>& r, const StepCoef<T>& q) -> T {
        T s = r.f;
        if constexpr (SHIFT)
            s += q.tl * (from_below(r.w, r.c) + from_above(r.w, r.c)) + q.ts * r.s + q.tn * r.n;
        else if constexpr (HAS_X)
            s += q.tl * (r.w + r.e) + q.ts * r.s + q.tn * r.n;
        return s;
    };

    Raw<T> rb[2][D];
    // the per-cell loads of chunk c, raw (combined when the chunk is solved)
    auto load = [&](const SegData<T>& sd, int c, int buf) {
#pragma unroll
        for (int d = 0; d < D; ++d) rb[buf][d] = fetch(sd, c * D + d);
    };
    // the half-column's forward values and couplings, by step
    T y[NS], cb[NS];
    // the old iterate of the half-column (KX), kept in LDS by step: the
    // registers hold the forward values and couplings
    __shared__ T xkl[KX ? 2 * kSweepPairs : 1][KX ? NS : 1][64];
    T(*xk)[64] = xkl[KX ? int(threadIdx.x >> 6) : 0];
    struct Fwd {
        T vp, cv, cprev, sm, im;
    };

    // Forward elimination of chunk c of a segment (its loads in rb[c & 1],
    // its step records in qb); vp: y of the last elimination step, cv: its
    // coupling times y (the wavefront's term of the meeting equation).
    auto fwd_chunk = [&](int c, const StepCoef<T>* qb, Fwd& st) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int t = c * D + d, sl = t;
            const StepCoef<T> q = qb[d];
            const Raw<T>& r = rb[c & 1][d];
            const T s = comb(r, q), ip = r.ip;
            if constexpr (KX) xk[sl][lane] = r.c;
            const T v = (s + st.cprev * st.vp) * ip;
            y[sl] = v;
            cb[sl] = q.tc * ip;
            // keep the coupling itself in a vector register: otherwise the
            // compiler keeps ip and the scalar tc of every step and spills
            // the scalars
            asm volatile("" : "+v"(cb[sl]));
            const bool elim = t < (top ? TM : M);
            if (top && t == TM) {
                st.sm = s;
                st.im = ip;
            }
            st.cv = elim ? q.tc * v : st.cv;
            st.vp = elim ? v : st.vp;
            st.cprev = q.tc;
        }
    };
    auto records = [&](const SegData<T>& sd, int c, StepCoef<T>* qb) {
#pragma unroll
        for (int d = 0; d < D; ++d) qb[d] = step_rec(sd.cr, c * D + d);
    };

    // meeting layer: x_m = (s_m + Tr_m y_{m-1} + Tr_{m+1} y_{m+1}) / d_m
    auto meet = [&](const Fwd& st) -> T {
        T(*xc)[64] = xch[p.pair];
        if (!top) {
            xc[0][lane] = st.cv;
        } else {
            xc[1][lane] = st.cv;
            xc[2][lane] = st.sm;
            xc[3][lane] = st.im;
        }
        __syncthreads();
        return (xc[2][lane] + xc[0][lane] + xc[1][lane]) * xc[3][lane];
    };

    // Back-substitution of chunk c (its steps from the last to the first)
    // of a segment from its meeting value xm, stored to xout; z carries the
    // solution of the step before. Without KX the old iterate of the chunk
    // is in xo[c & 1]. The layer offsets are formed again from an opaque
    // copy of the stride, not kept in scalar registers from the forward
    // pass.
    T xo[2][KX || !HAS_X ? 1 : D];
    auto bwd_chunk = [&](const SegData<T>& sd, int c, T xm, T& z) {
        uint32_t Pb2 = Pb;
        asm volatile("" : "+s"(Pb2));
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const int t = c * D + d, sl = t;
            const bool own = t < (top ? TM + 1 : M);
            const T zt = (top && t == TM) ? xm : y[sl] + cb[sl] * z;
            z = own ? zt : z;
            T out = omega * z;
            if constexpr (KX) out += keep * xk[sl][lane];
            else if constexpr (HAS_X) out += keep * xo[c & 1][d];
            int k = top ? nz - 1 - t : t;
            k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
            if (own && (FULL || sd.valid)) bst<NT_STORE>(out, ro, sd.oc, uint32_t(k) * Pb2);
        }
    };
    auto load_x = [&](const SegData<T>& sd, int c, int buf) {
        if constexpr (HAS_X && !KX) {
#pragma unroll
            for (int d = 0; d < D; ++d) xo[buf][d] = bld<T>(rx, sd.oc, soff(c * D + d));
        }
    };
    // the whole back-substitution of a segment (no other work beside it)
    auto bwd_all = [&](const SegData<T>& sd, T xm) {
        T z = xm;
        load_x(sd, NC - 1, (NC - 1) & 1);
#pragma unroll
        for (int c = NC - 1; c >= 0; --c) {
            if (c > 0) load_x(sd, c - 1, (c - 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
            bwd_chunk(sd, c, xm, z);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // forward elimination, the meeting exchange, back-substitution
    const SegData<T> sd(L, int(logical_block()), p.pair, top, wpr);
    asm volatile("" : "+s"(Pbi));
    Fwd st{T(0), T(0), T(0), T(0), T(0)};
    load(sd, 0, 0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        StepCoef<T> qb[D];
        records(sd, c, qb);
        __builtin_amdgcn_sched_barrier(0);
        if (c + 1 < NC) load(sd, c + 1, (c + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
        fwd_chunk(c, qb, st);
        __builtin_amdgcn_sched_barrier(0);
    }
    bwd_all(sd, meet(st));
}

}  // namespace

// Its addressing needs every per-cell array of the level below 4 GiB
// (grids are limited to fewer than 2^29 cells).
template <typename T>
void sweep(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega, hipStream_t s) {
    const int wpr = segments_per_row(L.nI);
    constexpr int threads = 128 * kSweepPairs;
    const bool full = L.nI % 64 == 0 && L.nJ % kSweepPairs == 0;
    using F = std::false_type;
    using Tt = std::true_type;
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    auto go = [&](auto nzc, auto exc, auto fullc, auto cpc) {
        constexpr int NZ = decltype(nzc)::value;
        constexpr bool EX = decltype(exc)::value, FULL = decltype(fullc)::value;
        constexpr int CP = decltype(cpc)::value;
        const int nb = tiled_blocks(L.nJ, wpr, kSweepPairs);
        if (xin)
            k_sweep<T, NZ, EX, FULL, true, CP>
                <<<nb, threads, 0, s>>>(L, f, xin, xout, omega, wpr);
        else
            k_sweep<T, NZ, EX, FULL, false, CP>
                <<<nb, threads, 0, s>>>(L, f, xin, xout, omega, wpr);
    };
    // the workloads' layer counts (70 and 16) exactly, others in buckets;
    // the non-temporal hints on large full levels of those counts
    const long long cells = L.plane * L.nz;
    auto exact = [&](auto nzc) {
        if (!full) go(nzc, Tt{}, F{}, P0{});
        else if (cells * (long long)sizeof(T) >= kStreamFieldBytes) go(nzc, Tt{}, Tt{}, P2{});
        else if (cells >= kSweepStreamCells) go(nzc, Tt{}, Tt{}, P1{});
        else go(nzc, Tt{}, Tt{}, P0{});
    };
    if (L.nz == 70) exact(std::integral_constant<int, 70>{});
    else if (L.nz == 16) exact(std::integral_constant<int, 16>{});
    else with_nz(L.nz, [&](auto nzc) { go(nzc, F{}, F{}, P0{}); });
}

template void sweep<float>(const LevelView<float>&, const float*, const float*, float*, float,
                           hipStream_t);
template void sweep<double>(const LevelView<double>&, const double*, const double*, double*,
                            double, hipStream_t);

}  // namespace mgk
