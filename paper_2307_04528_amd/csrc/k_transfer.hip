// Grid transfers of the horizontal-only hierarchy (paper Sections 2, 2.2):
//   restriction R: sum over the children (2 longitudes x 1 or 2 rows), fused
//                  with the residual f - H x (the paper restricts the residual);
//   prolongation P: cell-centred bilinear interpolation;
// and, for the transposed V-cycle, P^T and the transpose of the fused
// residual restriction.
#include "device.hpp"

namespace mgk {

namespace {
using namespace dev;

// Rows per block of the one-lane-per-cell kernels (64 columns x this many
// rows of one layer: each wavefront one row).
constexpr int kRowsPerBlock = 4;

// Two adjacent values (the two longitude children of a coarse column).
template <typename T>
__device__ __forceinline__ pair_t<T> ld2(gcptr base, uint32_t boff) {
    return *(const __attribute__((address_space(1))) pair_t<T>*)(base + boff);
}

// fc = R (f - H x), one wavefront per (row-aligned coarse segment, chunk of
// DL layers), chunk-major. A lane owns one coarse column: its
// two longitude children are adjacent, so each child row is one 2-value load;
// the children rows, tables and transfer maps are wave-uniform. The x values
// of the chunk's layers and the layers just outside it are loaded once.
// Chunk depth: 7 layers for FP32 on large levels (7 divides the 70-layer
// workloads: 185 us per finest-level launch on 1024x768x70, against 199 us
// with 4 layers, 190 with 6 and 212 with 8); 4 elsewhere (smaller levels
// need the parallelism of more chunks, and FP64 solves were 5 % slower with 7).
constexpr int kRestrictLayers = 4;
constexpr int kRestrictLayersLarge32 = 7;
template <typename T, bool HAS_X, int DL>
__global__ __launch_bounds__(kBlock) void k_restrict_seg(LevelView<T> F, TransferView<T> X,
                                                         const T* __restrict__ f,
                                                         const T* __restrict__ x,
                                                         T* __restrict__ fc, int wprc, int nsegc,
                                                         int units) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int unit = int(logical_block()) * (kBlock / 64) + wave;
    if (unit >= units) return;   // wave-uniform
    const int ch = unit / nsegc, seg = unit - ch * nsegc;
    const Seg gc = segment(seg, X.nIc, X.nJc, wprc);
    const int nI = F.nI, nJ = F.nJ, nz = F.nz;
    const int Jc = gc.J, Ic = int(gc.c) - Jc * X.nIc;
    const int j0 = tab(X.child_first, Jc);
    const int two = tab(X.child_count, Jc) - 1;   // 0 or 1
    const int j1 = j0 + two;
    const T w1 = T(two);
    constexpr uint32_t S = sizeof(T);
    const uint32_t i0 = 2 * uint32_t(Ic), i1 = i0 + 1;
    const uint32_t iw = (i0 == 0) ? uint32_t(nI - 1) : i0 - 1;
    const uint32_t ie = (i1 == uint32_t(nI - 1)) ? 0u : i1 + 1;
    const uint32_t r0 = uint32_t(j0) * nI, r1 = uint32_t(j1) * nI;
    const uint32_t rs = (j0 > 0) ? r0 - nI : r0, rn = (j1 < nJ - 1) ? r1 + nI : r1;
    const uint32_t o0 = (r0 + i0) * S, o1 = (r1 + i0) * S;
    const uint64_t Pb = uint64_t(F.plane) * S, Pcb = uint64_t(X.nIc) * X.nJc * S;
    const uint32_t oc = gc.c * S;
    const int k0 = ch * DL;
    T out[DL];
    if constexpr (!HAS_X) {
#pragma unroll
        for (int d = 0; d < DL; ++d) {
            gcptr fk = layer(f, clampk(k0 + d, nz), Pb);
            const pair_t<T> a = ld2<T>(fk, o0), b = ld2<T>(fk, o1);
            out[d] = a.x + a.y + w1 * (b.x + b.y);
        }
    } else {
        const uint32_t ow0 = (r0 + iw) * S, oe0 = (r0 + ie) * S, ow1 = (r1 + iw) * S,
                       oe1 = (r1 + ie) * S, os = (rs + i0) * S, on = (rn + i0) * S;
        // children of the layers k0-1 .. k0+DL (clamped; the vertical couplings
        // are 0 at the bottom and top)
        pair_t<T> c0[DL + 2], c1[DL + 2];
#pragma unroll
        for (int d = 0; d < DL + 2; ++d) {
            const int kk = k0 - 1 + d;
            gcptr xk = layer(x, kk < 0 ? 0 : clampk(kk, nz), Pb);
            c0[d] = ld2<T>(xk, o0);
            c1[d] = ld2<T>(xk, o1);
        }
#pragma unroll
        for (int d = 0; d < DL; ++d) {
            const int kk = clampk(k0 + d, nz);
            gcptr fk = layer(f, kk, Pb), Mk = layer(F.M, kk, Pb), xk = layer(x, kk, Pb);
            const pair_t<T> fa = ld2<T>(fk, o0), fb = ld2<T>(fk, o1);
            const pair_t<T> ma = ld2<T>(Mk, o0), mb = ld2<T>(Mk, o1);
            const pair_t<T> xs = ld2<T>(xk, os), xn = ld2<T>(xk, on);
            const T xw0 = ldb<T>(xk, ow0), xe0 = ldb<T>(xk, oe0), xw1 = ldb<T>(xk, ow1),
                    xe1 = ldb<T>(xk, oe1);
            const pair_t<T> a = c0[d + 1], b = c1[d + 1];
            const pair_t<T> am = c0[d], bm = c1[d], ap = c0[d + 2], bp = c1[d + 2];
            const T tl0 = tab(F.Tlam, kk * nJ + j0), tl1 = tab(F.Tlam, kk * nJ + j1);
            const T ts0 = tab(F.Tth, kk * (nJ + 1) + j0), tn0 = tab(F.Tth, kk * (nJ + 1) + j0 + 1);
            const T ts1 = tab(F.Tth, kk * (nJ + 1) + j1), tn1 = tab(F.Tth, kk * (nJ + 1) + j1 + 1);
            const T tb0 = tab(F.Tr, kk * nJ + j0), tt0 = tab(F.Tr, (kk + 1) * nJ + j0);
            const T tb1 = tab(F.Tr, kk * nJ + j1), tt1 = tab(F.Tr, (kk + 1) * nJ + j1);
            // a merged row's other row is its latitude neighbour
            const T n00 = two ? b.x : xn.x, n01 = two ? b.y : xn.y;
            const T s10 = two ? a.x : xs.x, s11 = two ? a.y : xs.y;
            const T h0 = ma.x * a.x + hdiff(tl0, ts0, tn0, a.x, xw0, a.y, xs.x, n00) +
                         ma.y * a.y + hdiff(tl0, ts0, tn0, a.y, a.x, xe0, xs.y, n01) +
                         tb0 * ((a.x - am.x) + (a.y - am.y)) + tt0 * ((a.x - ap.x) + (a.y - ap.y));
            const T h1 = mb.x * b.x + hdiff(tl1, ts1, tn1, b.x, xw1, b.y, s10, xn.x) +
                         mb.y * b.y + hdiff(tl1, ts1, tn1, b.y, b.x, xe1, s11, xn.y) +
                         tb1 * ((b.x - bm.x) + (b.y - bm.y)) + tt1 * ((b.x - bp.x) + (b.y - bp.y));
            out[d] = fa.x + fa.y + w1 * (fb.x + fb.y) - (h0 + w1 * h1);
        }
    }
#pragma unroll
    for (int d = 0; d < DL; ++d)
        if (k0 + d < nz && gc.valid) stb<T>(layer_w(fc, k0 + d, Pcb), oc, out[d]);
}

// fc = R (f - H x) on the larger levels (see RestrictWalk), whose step
// records cover every layer (nz <= kStepStride). One wavefront per (row-aligned coarse
// segment, range of LR layers), range-major, walks its layers upward with
// the loads of the next P layers in flight. The children of a layer serve
// as the layer above of the step before and the layer below of the step
// after, so each is loaded once (and one layer below the range). A lane
// loads, per layer, its two children in each child row (one 2-value load
// each), the rows south and north of the children, its four longitude
// neighbours, f and the mass; a row's couplings are its upward step record
// (Tlam, Ttheta south and north, Tr above), Tr below being the record of
// the layer before.
// Per precision: layers per range, layers in flight ahead, waves per SIMD,
// and the smallest level (columns) that walks. FP32 on 1024x768x70, per
// finest-level launch: 171 us with ranges of 10 layers, 175 with 14, 178
// with 35; on 384x192x70 (73,728 columns) 21 us against 24 us for the
// chunked kernel, and the whole solve 0.1-0.2 ms faster on both shells.
// FP64: 303 us with ranges of 10 layers against 320 us with 14 or 35.
template <typename T>
struct RestrictWalk;
template <>
struct RestrictWalk<float> {
    static constexpr int LR = 10, P = 3, W = 4;
    static constexpr long long MinColumns = 1LL << 15;
};
template <>
struct RestrictWalk<double> {
    static constexpr int LR = 10, P = 2, W = 2;
    static constexpr long long MinColumns = 1LL << 15;
};
// FULLI: every segment has 64 coarse columns (nIc a multiple of 64); then a
// lane's longitude neighbours are its neighbour lanes' children, and only
// lanes 0 and 63 load theirs (one load per child row).
// NTL: f and the mass loaded with the non-temporal hint (fields of at least
// kStreamFieldBytes).
template <typename T, int LR, int P, int W, bool FULLI, bool NTL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(W)))
void k_restrict_walk(LevelView<T> F, TransferView<T> X, const T* __restrict__ f,
                     const T* __restrict__ x, T* __restrict__ fc, int wprc, int nsegc,
                     int units) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int unit = int(logical_block()) * (kBlock / 64) + wave;
    if (unit >= units) return;   // wave-uniform
    const int rg = unit / nsegc, seg = unit - rg * nsegc;
    const Seg gc = segment(seg, X.nIc, X.nJc, wprc);
    const int nI = F.nI, nJ = F.nJ, nz = F.nz;
    const int Jc = gc.J, Ic = int(gc.c) - Jc * X.nIc;
    const int j0 = tab(X.child_first, Jc);
    const int two = tab(X.child_count, Jc) - 1;   // 0 or 1
    const int j1 = j0 + two;
    const T w1 = T(two);
    constexpr uint32_t S = sizeof(T);
    const uint32_t i0 = 2 * uint32_t(Ic), i1 = i0 + 1;
    const uint32_t iw = (i0 == 0) ? uint32_t(nI - 1) : i0 - 1;
    const uint32_t ie = (i1 == uint32_t(nI - 1)) ? 0u : i1 + 1;
    const uint32_t r0 = uint32_t(j0) * nI, r1 = uint32_t(j1) * nI;
    const uint32_t rs = (j0 > 0) ? r0 - nI : r0, rn = (j1 < nJ - 1) ? r1 + nI : r1;
    const uint32_t o0 = (r0 + i0) * S, o1 = (r1 + i0) * S, os = (rs + i0) * S,
                   on = (rn + i0) * S;
    const uint32_t ow0 = (r0 + iw) * S, oe0 = (r0 + ie) * S, ow1 = (r1 + iw) * S,
                   oe1 = (r1 + ie) * S;
    // lane 0 loads the west edge, lane 63 the east edge, other lanes their
    // east neighbour (a cache hit; unused)
    const bool lane0 = (threadIdx.x & 63u) == 0;
    const uint32_t og0 = lane0 ? ow0 : oe0, og1 = lane0 ? ow1 : oe1;
    const uint32_t Pb = uint32_t(F.plane) * S, Pcb = uint32_t(X.nIc) * uint32_t(X.nJc) * S;
    const rsrc_t rx = make_rsrc(x, Pb * uint32_t(nz)), rf = make_rsrc(f, Pb * uint32_t(nz)),
                 rm = make_rsrc(F.M, Pb * uint32_t(nz)), ro = make_rsrc(fc, Pcb * uint32_t(nz));
    const StepCoef<T>* q0p = F.sc + size_t(j0) * kStepStride;
    const StepCoef<T>* q1p = F.sc + size_t(j1) * kStepStride;
    const uint32_t oc = gc.c * S;
    const int kb = rg * LR;

    struct Lay {
        pair_t<T> a, b, xs, xn, fa, fb, ma, mb;
        T w0, e0, w1, e1;
        StepCoef<T> q0, q1;
    };
    // the loads of step t (layer kb + t, clamped) with its step records;
    // only the children for the layer above the range
    auto fetch = [&](int t, bool children_only) {
        Lay L;
        const int k = clampk(kb + t, nz);
        const uint32_t so = uint32_t(k) * Pb;
        L.a = bld2<T>(rx, o0, so);
        L.b = bld2<T>(rx, o1, so);
        if (!children_only) {
            L.xs = bld2<T>(rx, os, so);
            L.xn = bld2<T>(rx, on, so);
            if constexpr (FULLI) {
                L.w0 = bld<T>(rx, og0, so);   // the edges of the segment's rows
                L.w1 = bld<T>(rx, og1, so);
            } else {
                L.w0 = bld<T>(rx, ow0, so);
                L.e0 = bld<T>(rx, oe0, so);
                L.w1 = bld<T>(rx, ow1, so);
                L.e1 = bld<T>(rx, oe1, so);
            }
            // f and the mass are read at the children only
            L.fa = bld2<T, NTL>(rf, o0, so);
            L.fb = bld2<T, NTL>(rf, o1, so);
            L.ma = bld2<T, NTL>(rm, o0, so);
            L.mb = bld2<T, NTL>(rm, o1, so);
            L.q0 = step_rec(q0p, size_t(k));
            L.q1 = step_rec(q1p, size_t(k));
        }
        return L;
    };

    // the layer below the range, and its vertical couplings to the first
    // layer (0 at the bottom)
    const int kbm = kb > 0 ? kb - 1 : 0;
    pair_t<T> am = bld2<T>(rx, o0, uint32_t(kbm) * Pb), bm = bld2<T>(rx, o1, uint32_t(kbm) * Pb);
    const T tbm0 = step_rec(q0p, size_t(kbm)).tc, tbm1 = step_rec(q1p, size_t(kbm)).tc;
    T tb0 = kb > 0 ? tbm0 : T(0), tb1 = kb > 0 ? tbm1 : T(0);
    Lay buf[P + 1];
#pragma unroll
    for (int t = 0; t < P; ++t) {
        __builtin_amdgcn_sched_barrier(0);
        buf[t] = fetch(t, t == LR);
    }
#pragma unroll
    for (int t = 0; t < LR; ++t) {
        __builtin_amdgcn_sched_barrier(0);
        if (t + P <= LR) buf[(t + P) % (P + 1)] = fetch(t + P, t + P == LR);
        __builtin_amdgcn_sched_barrier(0);
        const Lay& c = buf[t % (P + 1)];
        const pair_t<T> ap = buf[(t + 1) % (P + 1)].a, bp = buf[(t + 1) % (P + 1)].b;
        const StepCoef<T> q0 = c.q0, q1 = c.q1;
        const pair_t<T> a = c.a, b = c.b, xs = c.xs, xn = c.xn;
        T w0, e0, w1v, e1;
        if constexpr (FULLI) {
            w0 = from_below(c.w0, a.y);
            e0 = from_above(c.w0, a.x);
            w1v = from_below(c.w1, b.y);
            e1 = from_above(c.w1, b.x);
        } else {
            w0 = c.w0;
            e0 = c.e0;
            w1v = c.w1;
            e1 = c.e1;
        }
        // a merged row's other row is its latitude neighbour
        const T n00 = two ? b.x : xn.x, n01 = two ? b.y : xn.y;
        const T s10 = two ? a.x : xs.x, s11 = two ? a.y : xs.y;
        const T h0 = c.ma.x * a.x + hdiff(q0.tl, q0.ts, q0.tn, a.x, w0, a.y, xs.x, n00) +
                     c.ma.y * a.y + hdiff(q0.tl, q0.ts, q0.tn, a.y, a.x, e0, xs.y, n01) +
                     tb0 * ((a.x - am.x) + (a.y - am.y)) +
                     q0.tc * ((a.x - ap.x) + (a.y - ap.y));
        const T h1 = c.mb.x * b.x + hdiff(q1.tl, q1.ts, q1.tn, b.x, w1v, b.y, s10, xn.x) +
                     c.mb.y * b.y + hdiff(q1.tl, q1.ts, q1.tn, b.y, b.x, e1, s11, xn.y) +
                     tb1 * ((b.x - bm.x) + (b.y - bm.y)) +
                     q1.tc * ((b.x - bp.x) + (b.y - bp.y));
        T out = c.fa.x + c.fa.y + w1 * (c.fb.x + c.fb.y) - (h0 + w1 * h1);
        // computed here, not sunk (with its loads) into the guarded store
        asm volatile("" : "+v"(out));
        if (kb + t < nz && gc.valid) bst(out, ro, oc, uint32_t(kb + t) * Pcb);
        am = a;
        bm = b;
        tb0 = q0.tc;
        tb1 = q1.tc;
    }
}

// x += P xc: bilinear interpolation (3/4, 1/4 in longitude; the row weights
// of the map in latitude). One wavefront per (row-aligned segment, chunk of
// prolong_layers<T>() layers), chunk-major so that each XCD streams a band of rows
// of one chunk: the fine row's coarse rows and weights are wave-uniform, the
// per-lane coarse columns are computed once, and the loads of the whole chunk
// are independent and issued together.
// (FP32 8: 98 us on 1024x768x70, against 115 us with 4 or 16 layers)
constexpr int kProlongLayers = 8;
// FP64: 2 layers (245 us against 262 us with 8 and 291 us with 16 on
// 1024x768x70; its loads take twice the registers)
template <typename T>
constexpr int prolong_layers() {
    return std::is_same<T, float>::value ? kProlongLayers : 2;
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelView<T> F, TransferView<T> X,
                                                        const T* __restrict__ xc,
                                                        T* __restrict__ x, int wpr, int nseg,
                                                        int units) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int unit = int(logical_block()) * (kBlock / 64) + wave;
    if (unit >= units) return;   // wave-uniform
    const int ch = unit / nseg, seg = unit - ch * nseg;
    const Seg g = segment(seg, F.nI, F.nJ, wpr);
    const int j = g.J, i = int(g.c) - j * F.nI, nIc = X.nIc;
    const int J0 = tab(X.prow, 2 * j), J1 = tab(X.prow, 2 * j + 1);
    const T w0 = tab(X.pw, 2 * j), w1 = tab(X.pw, 2 * j + 1);
    const int I = i >> 1;
    const int In = (i & 1) ? (I + 1 == nIc ? 0 : I + 1) : (I == 0 ? nIc - 1 : I - 1);
    constexpr uint32_t S = sizeof(T);
    const uint32_t o0 = uint32_t(J0 * nIc + I) * S, o0n = uint32_t(J0 * nIc + In) * S;
    const uint32_t o1 = uint32_t(J1 * nIc + I) * S, o1n = uint32_t(J1 * nIc + In) * S;
    const uint32_t ox = g.c * S;
    const uint64_t Pb = uint64_t(F.plane) * S, Pcb = uint64_t(nIc) * X.nJc * S;
    constexpr int NL = prolong_layers<T>();
    const int nz = F.nz, k0 = ch * NL;
    const T a = T(0.75), b = T(0.25);
    T v[NL];
#pragma unroll
    for (int d = 0; d < NL; ++d) {
        const int kk = clampk(k0 + d, nz);
        gcptr ck = layer(xc, kk, Pcb);
        v[d] = ldb<T>(layer(x, kk, Pb), ox) + w0 * (a * ldb<T>(ck, o0) + b * ldb<T>(ck, o0n)) +
               w1 * (a * ldb<T>(ck, o1) + b * ldb<T>(ck, o1n));
    }
#pragma unroll
    for (int d = 0; d < NL; ++d)
        if (k0 + d < nz && g.valid) stb<T>(layer_w(x, k0 + d, Pb), ox, v[d]);
}

// Layers per lane of the transposed transfers (a lane walks a chunk of
// layers of its column, the chunk's loads in flight together).
// (P^T: 2; FP32 adjoint solves on 1024x768x70 1.2 % slower with 4, 2.2 %
// with 8)
template <typename T>
constexpr int prolong_T_layers() {
    return 2;
}
constexpr int kInjectLayers = 8;

// xc = P^T x, one lane per coarse column and chunk of prolong_T_layers layers.
// A coarse column I gathers fine columns 2I-1 .. 2I+2 of up to four fine
// rows. Each lane loads its own two (2I, 2I+1) as one pair; the outer two
// are its neighbour lanes' (shuffled), except at the edges of the
// wavefront's 64 columns, whose two values are wave-uniform loads. Every
// lane stays active for the shuffles: lanes past the row's end compute on
// the last column and store nothing.
template <typename T>
__global__ __launch_bounds__(64 * kRowsPerBlock) void k_prolong_T(LevelView<T> F,
                                                                  TransferView<T> X,
                                                                  const T* __restrict__ x,
                                                                  T* __restrict__ xc) {
    constexpr int NL = prolong_T_layers<T>();
    using V2 = std::conditional_t<std::is_same<T, float>::value, float2, double2>;
    // blocks of 64 coarse columns x kRowsPerBlock coarse rows
    const int lane = int(threadIdx.x);
    const int Ic0 = int(blockIdx.x) * 64, nIc = X.nIc;
    const int Jc = __builtin_amdgcn_readfirstlane(int(blockIdx.y) * kRowsPerBlock +
                                                  int(threadIdx.y));
    const int k0 = int(blockIdx.z) * NL, nz = F.nz;
    if (Jc >= X.nJc) return;   // wave-uniform
    const int nIf = F.nI;
    const bool valid = Ic0 + lane < nIc;
    const int iE = 2 * (valid ? Ic0 + lane : nIc - 1);
    // the wavefront's last column, and the fine columns west of its first
    // and east of its last (wrapping around the circle of longitude)
    const int lastl = (nIc - Ic0 < 64 ? nIc - Ic0 : 64) - 1;
    const int iW0 = (Ic0 == 0) ? nIf - 1 : 2 * Ic0 - 1;
    const int iEE1 = (Ic0 + lastl + 1 == nIc) ? 0 : 2 * (Ic0 + lastl) + 2;
    const T a = T(0.75), b = T(0.25);
    size_t roff[4];
    T wr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = X.ptrow[4 * Jc + e];
        roff[e] = size_t(row < 0 ? 0 : row) * nIf;
        wr[e] = X.ptw[4 * Jc + e];
    }
    T acc[NL];
#pragma unroll
    for (int d = 0; d < NL; ++d) {
        const int k = k0 + d < nz ? k0 + d : nz - 1;
        acc[d] = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const T* r = x + size_t(k) * F.plane + roff[e];
            const V2 p = *reinterpret_cast<const V2*>(r + iE);
            const T w0 = r[iW0], e1 = r[iEE1];
            T rw = __shfl_up(p.y, 1, 64);
            T ree = __shfl_down(p.x, 1, 64);
            if (lane == 0) rw = w0;
            if (lane == lastl) ree = e1;
            acc[d] += wr[e] * (a * (p.x + p.y) + b * (rw + ree));
        }
    }
    const size_t Pc = size_t(nIc) * X.nJc;
    const size_t cc = size_t(Jc) * nIc + size_t(Ic0 + lane);
#pragma unroll
    for (int d = 0; d < NL; ++d)
        if (valid && k0 + d < nz) xc[size_t(k0 + d) * Pc + cc] = acc[d];
}

// x += R^T xc (every child takes its coarse value), one lane per fine
// column and chunk of kInjectLayers layers, in blocks of 64 columns x
// kRowsPerBlock rows (the row's coarse row wave-uniform).
template <typename T>
__global__ __launch_bounds__(64 * kRowsPerBlock) void k_inject_add(LevelView<T> F,
                                                                   TransferView<T> X,
                                                                   const T* __restrict__ xc,
                                                                   T* __restrict__ x) {
    constexpr int NL = kInjectLayers;
    const int nI = F.nI, nJ = F.nJ, nIc = X.nIc, nz = F.nz;
    const int i = int(blockIdx.x) * 64 + int(threadIdx.x);
    const int j = __builtin_amdgcn_readfirstlane(int(blockIdx.y) * kRowsPerBlock +
                                                 int(threadIdx.y));
    const int k0 = int(blockIdx.z) * NL;
    if (i >= nI || j >= nJ) return;
    const size_t P = size_t(F.plane), Pc = size_t(nIc) * X.nJc;
    const size_t c = size_t(j) * size_t(nI) + size_t(i);
    const size_t cc = size_t(X.crow_of[j]) * size_t(nIc) + size_t(i >> 1);
    T v[NL];
#pragma unroll
    for (int d = 0; d < NL; ++d) {
        const int k = k0 + d < nz ? k0 + d : nz - 1;
        v[d] = x[size_t(k) * P + c] + xc[size_t(k) * Pc + cc];
    }
#pragma unroll
    for (int d = 0; d < NL; ++d)
        if (k0 + d < nz) x[size_t(k0 + d) * P + c] = v[d];
}

}  // namespace

template <typename T>
void restrict_residual(const LevelView<T>& F, const TransferView<T>& X, const T* f,
                       const T* x, T* fc, hipStream_t s) {
    const int wprc = segments_per_row(X.nIc);
    const int nsegc = X.nJc * wprc;
    constexpr int waves = kBlock / 64;
    constexpr int DLS = kRestrictLayers;
    constexpr int DLL = std::is_same<T, float>::value ? kRestrictLayersLarge32 : DLS;
    if (x && F.plane >= RestrictWalk<T>::MinColumns && F.nz <= kStepStride) {
        using C = RestrictWalk<T>;
        const int units = nsegc * ((F.nz + C::LR - 1) / C::LR);
        const int nb = (units + waves - 1) / waves;
        auto go = [&](auto fulli, auto ntl) {
            k_restrict_walk<T, C::LR, C::P, C::W, decltype(fulli)::value, decltype(ntl)::value>
                <<<nb, kBlock, 0, s>>>(F, X, f, x, fc, wprc, nsegc, units);
        };
        using Tt = std::true_type;
        using Ff = std::false_type;
        const bool ntl = F.plane * F.nz * (long long)sizeof(T) >= kStreamFieldBytes;
        if (X.nIc % 64 == 0) {
            if (ntl) go(Tt{}, Tt{});
            else go(Tt{}, Ff{});
        } else {
            if (ntl) go(Ff{}, Tt{});
            else go(Ff{}, Ff{});
        }
    } else if (F.plane >= kSmallLevelColumns) {
        const int units = nsegc * ((F.nz + DLL - 1) / DLL);
        const int nb = (units + waves - 1) / waves;
        if (x) k_restrict_seg<T, true, DLL><<<nb, kBlock, 0, s>>>(F, X, f, x, fc, wprc, nsegc, units);
        else k_restrict_seg<T, false, DLL><<<nb, kBlock, 0, s>>>(F, X, f, x, fc, wprc, nsegc, units);
    } else {
        const int units = nsegc * ((F.nz + DLS - 1) / DLS);
        const int nb = (units + waves - 1) / waves;
        if (x) k_restrict_seg<T, true, DLS><<<nb, kBlock, 0, s>>>(F, X, f, x, fc, wprc, nsegc, units);
        else k_restrict_seg<T, false, DLS><<<nb, kBlock, 0, s>>>(F, X, f, x, fc, wprc, nsegc, units);
    }
}

template <typename T>
void prolong_add(const LevelView<T>& F, const TransferView<T>& X, const T* xc, T* x,
                 hipStream_t s) {
    const int wpr = segments_per_row(F.nI);
    const int nseg = F.nJ * wpr;
    constexpr int NL = prolong_layers<T>();
    const int units = nseg * ((F.nz + NL - 1) / NL);
    constexpr int waves = kBlock / 64;
    k_prolong_add<T><<<(units + waves - 1) / waves, kBlock, 0, s>>>(F, X, xc, x, wpr, nseg,
                                                                    units);
}

template <typename T>
void prolong_transpose(const LevelView<T>& F, const TransferView<T>& X, const T* x, T* xc,
                       hipStream_t s) {
    const dim3 grid(unsigned((X.nIc + 63) / 64),
                    unsigned((X.nJc + kRowsPerBlock - 1) / kRowsPerBlock),
                    unsigned((F.nz + prolong_T_layers<T>() - 1) / prolong_T_layers<T>()));
    k_prolong_T<T><<<grid, dim3(64, kRowsPerBlock), 0, s>>>(F, X, x, xc);
}

template <typename T>
void inject_add(const LevelView<T>& F, const TransferView<T>& X, const T* xc, T* x,
                hipStream_t s) {
    const dim3 grid(unsigned((F.nI + 63) / 64), unsigned((F.nJ + kRowsPerBlock - 1) / kRowsPerBlock),
                    unsigned((F.nz + kInjectLayers - 1) / kInjectLayers));
    k_inject_add<T><<<grid, dim3(64, kRowsPerBlock), 0, s>>>(F, X, xc, x);
}

#define MG_INST(T)                                                                       \
    template void restrict_residual<T>(const LevelView<T>&, const TransferView<T>&,      \
                                       const T*, const T*, T*, hipStream_t);              \
    template void prolong_add<T>(const LevelView<T>&, const TransferView<T>&, const T*,  \
                                 T*, hipStream_t);                                        \
    template void prolong_transpose<T>(const LevelView<T>&, const TransferView<T>&,      \
                                       const T*, T*, hipStream_t);                        \
    template void inject_add<T>(const LevelView<T>&, const TransferView<T>&, const T*, T*, \
                                hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

}  // namespace mgk
