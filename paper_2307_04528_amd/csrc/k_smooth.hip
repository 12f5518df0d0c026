// Block-Jacobi smoother (paper Eq. 1, Section 2.1) on the small and the
// coarsest levels, and its transpose (adjoint cycle).
//
// One sweep, with the vertical couplings in H_z solved exactly per column:
//   x_new = (1 - omega) x + omega H_z^{-1} (f + sum_h T_h x_nb)
// which equals x + omega H_z^{-1}(f - H x) since H = H_z + dH and dH holds
// only the horizontal off-diagonals -T_h. Levels that fill the GPU sweep
// with k_sweep (k_sweep.hip); the kernels here take the levels below
// staged_columns (k_smooth_staged), the coarsest level (k_coarse_lds,
// k_coarse_solve) and the transposed sweeps (k_smooth_T).
//
// Column solves use the twisted factorisation of H_z (pivots from setup). A
// pair of wavefronts takes one row-aligned segment of up to 64 columns: the
// bottom wavefront eliminates the layers below the meeting layer m = nz/2
// going up, the top wavefront the layers above it going down; after one
// exchange through LDS both know layer m, and each back-substitutes outward.
// A wavefront thus walks half a column: the chain of dependent steps is half
// as long as a one-sided Thomas solve.
#include "device.hpp"

namespace mgk {

namespace {
using namespace dev;

// Layers per prefetch chunk of the column kernels here.
template <typename T>
struct ChunkDepth {
    static constexpr int value = std::is_same<T, float>::value ? 6 : 2;
};

// Prefetch the raw loads of a chunk (FP64: the loads then stay in flight
// while the previous chunk is solved) or combine them into the chunk's
// right-hand sides at fetch time (FP32: fewer registers).
template <typename T>
struct RawPrefetch {
    static constexpr bool value = !std::is_same<T, float>::value;
};

// Read a wavefront's row couplings from lane tables (FP32) or with scalar
// loads (FP64: the tables' registers would spill the x sweep).
template <typename T>
struct LaneTables {
    static constexpr bool value = std::is_same<T, float>::value;
};

// Steps of one wavefront of a pair for the layer bucket NZ.
template <int NZ>
constexpr int half_steps() { return (NZ + 1) / 2; }
template <int NZ, int D>
constexpr int padded_steps() { return ((half_steps<NZ>() + D - 1) / D) * D; }

// Twisted solve z = H_z^{-1} s of one column by one wavefront of a pair.
//   top          : false for the bottom wavefront, true for the top (uniform)
//   xch          : 256 values of LDS private to the pair
//   fetch(t, kk) : issues the loads of layer kk (step t) and returns them
//                  raw (any struct), with no arithmetic on them, so that a
//                  chunk's loads stay in flight while the previous chunk is
//                  solved
//   comb(t, kk, raw): s_kk from the fetched values
//   inv(kk)      : the stored twisted pivot of layer kk
//   cpl(F)       : Tr_F, the vertical coupling across face F (below layer F)
//   fsink(t, kk, s): s of one of this wavefront's layers is available
//   bload(kk)    : (BL only) a per-layer value the back-substitution needs,
//                  loaded one chunk ahead like the forward loads
//   sink(t, kk, z, e): z of one of this wavefront's layers, from the meeting
//                    layer outward (the top wavefront owns layer m), with
//                    e = bload(kk) (0 without BL)
// Step t is layer t (bottom) or nz-1-t (top). Steps beyond a wavefront's
// layers compute on clamped data and reach neither fsink nor sink. Every
// thread of the block must call this (one block barrier inside).
template <typename T, int NZ, int D, bool BL, class Fetch, class Comb, class Inv, class Cpl,
          class FSink, class BLoad, class Sink>
__device__ __forceinline__ void twisted_column(int nz, bool top, T* xch, Fetch fetch, Comb comb,
                                               Inv inv, Cpl cpl, FSink fsink, BLoad bload,
                                               Sink sink) {
    constexpr int NP = padded_steps<NZ, D>();
    constexpr int NC = NP / D;
    using Raw = decltype(fetch(0, 0));
    const int m = nz >> 1, tm = nz - 1 - m;
    const int nrec = top ? tm : m;   // steps eliminated by this wavefront
    T y[NP], cb[NP];
    // RAW: buffer the fetched values and combine them when the chunk is
    // solved; otherwise combine at fetch time and buffer s (fewer registers)
    constexpr bool RAW = RawPrefetch<T>::value;
    Raw br[2][RAW ? D : 1];
    T bs[2][RAW ? 1 : D];
    T bp[2][D];
    auto lay = [&](int t) {
        const int k = top ? nz - 1 - t : t;
        return k < 0 ? 0 : (k < nz ? k : nz - 1);
    };
    auto load = [&](int c, int buf) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int t = c * D + d, kk = lay(t);
            if constexpr (RAW) br[buf][d] = fetch(t, kk);
            else bs[buf][d] = comb(t, kk, fetch(t, kk));
            bp[buf][d] = inv(kk);
        }
    };
    T vp = 0, sm = 0, im = 0;
    load(0, 0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c + 1 < NC) load(c + 1, (c + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int t = c * D + d, kk = lay(t);
            T s;
            if constexpr (RAW) s = comb(t, kk, br[c & 1][d]);
            else s = bs[c & 1][d];
            const T ip = bp[c & 1][d];
            if (t < nrec || (top && t == tm)) fsink(t, kk, s);
            // couplings to the layer eliminated before this one and to the
            // one after it
            const T cf = cpl(top ? kk + 1 : kk), cn = cpl(top ? kk : kk + 1);
            const T v = (s + cf * vp) * ip;
            y[t] = v;
            cb[t] = cn * ip;
            if (t == tm) {
                sm = s;
                im = ip;
            }
            vp = (t < nrec) ? v : vp;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    T be[2][BL ? D : 1];
    auto load_back = [&](int c, int buf) {
        if constexpr (BL) {
#pragma unroll
            for (int d = 0; d < D; ++d) be[buf][d] = bload(lay(c * D + d));
        }
    };
    load_back(NC - 1, (NC - 1) & 1);
    // meeting layer: x_m = (s_m + Tr_m y_{m-1} + Tr_{m+1} z_{m+1}) / d_m
    const int lane = int(threadIdx.x & 63u);
    if (!top) {
        xch[lane] = vp;
    } else {
        xch[64 + lane] = vp;
        xch[128 + lane] = sm;
        xch[192 + lane] = im;
    }
    __syncthreads();
    const T xm =
        (xch[128 + lane] + cpl(m) * xch[lane] + cpl(m + 1) * xch[64 + lane]) * xch[192 + lane];
    T xv = xm;
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
        if (BL && c > 0) load_back(c - 1, (c - 1) & 1);
        if constexpr (BL) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const int t = c * D + d, kk = lay(t);
            const T e = BL ? be[c & 1][BL ? d : 0] : T(0);
            if (top && t == tm) {
                sink(t, kk, xm, e);
            } else if (t < nrec) {
                xv = y[t] + cb[t] * xv;
                sink(t, kk, xv, e);
            }
        }
        if constexpr (BL) __builtin_amdgcn_sched_barrier(0);
    }
}

// The raw loads of one layer of a sweep: the right-hand side, and the
// iterate at the cell (c) and its four horizontal neighbours.
template <typename T>
struct StencilRaw {
    T f, c, w, e, s, n;
};

// The loads of one layer of a coarsest-level sweep: the stencil values and
// the row's horizontal couplings.
template <typename T>
struct CoarseRaw {
    T f, c, w, e, s, n, tl, ts, tn;
};

// Keep the old iterate of a column in registers between the two passes
// (FP32), or load it again in the back-substitution (FP64).
template <typename T>
struct KeepX {
    static constexpr bool value = std::is_same<T, float>::value;
};

// One sweep of the segment's columns (see the file comment); HAS_X false:
// the sweep from zero, omega H_z^{-1} f.
template <typename T, int NZ, int D, bool HAS_X>
__device__ __forceinline__ void sweep_segment(const LevelView<T>& L, const T* f, const T* xin,
                                              T* xout, T omega, const Seg& g, bool top,
                                              T* xch) {
    const NbB<T> b(g);
    const int nJ = L.nJ, J = g.J;
    const uint64_t Pb = uint64_t(L.plane) * sizeof(T);
    const T keep = T(1) - omega;
    constexpr bool KX = HAS_X && KeepX<T>::value;
    T xk[KX ? padded_steps<NZ, D>() : 1];
    auto fetch = [&](int, int kk) {
        StencilRaw<T> r{};
        r.f = ldb<T>(layer(f, kk, Pb), b.c);
        if constexpr (HAS_X) {
            gcptr xl = layer(xin, kk, Pb);
            r.w = ldb<T>(xl, b.w);
            r.e = ldb<T>(xl, b.e);
            r.s = ldb<T>(xl, b.s);
            r.n = ldb<T>(xl, b.n);
            if constexpr (KX) r.c = ldb<T>(xl, b.c);
        }
        return r;
    };
    // couplings of the row from lane tables (no memory wait per layer), or
    // through scalar loads where the registers are not there (FP64)
    constexpr bool LT = LaneTables<T>::value;
    using TabH = std::conditional_t<LT, LaneTable<T, NZ>, NoLaneTable<T>>;
    using TabV = std::conditional_t<LT, LaneTable<T, NZ + 1>, NoLaneTable<T>>;
    const int nzl = HAS_X ? L.nz : 0;
    const TabH tl(L.Tlam, nJ, J, nzl), ts(L.Tth, nJ + 1, J, nzl), tn(L.Tth, nJ + 1, J + 1, nzl);
    const TabV tr(L.Tr, nJ, J, L.nz + 1);
    auto comb = [&](int t, int kk, const StencilRaw<T>& r) -> T {
        T s = r.f;
        if constexpr (HAS_X) {
            if constexpr (LT)
                s += tl(kk) * (r.w + r.e) + ts(kk) * r.s + tn(kk) * r.n;
            else
                s += tab(L.Tlam, kk * nJ + J) * (r.w + r.e) +
                     tab(L.Tth, kk * (nJ + 1) + J) * r.s +
                     tab(L.Tth, kk * (nJ + 1) + J + 1) * r.n;
            if constexpr (KX) xk[t] = r.c;
        }
        return s;
    };
    auto cpl = [&](int F) -> T {
        if constexpr (LT) return tr(F);
        else return tab(L.Tr, F * nJ + J);
    };
    auto inv = [&](int kk) -> T { return ldb<T>(layer(L.invp, kk, Pb), b.c); };
    auto fsink = [](int, int, T) {};
    auto bload = [&](int kk) -> T { return ldb<T>(layer(xin, kk, Pb), b.c); };
    auto sink = [&](int t, int kk, T z, T e) {
        T out = omega * z;
        if constexpr (KX) out += keep * xk[t];
        else if constexpr (HAS_X) out += keep * e;
        if (g.valid) stb<T>(layer_w(xout, kk, Pb), b.c, out);
    };
    twisted_column<T, NZ, D, HAS_X && !KX>(L.nz, top, xch, fetch, comb, inv, cpl, fsink, bload,
                                            sink);
}

// ---------------------------------------------------------------------------
// Staged sweep for small levels. A level of a few thousand columns leaves
// most of the GPU idle: a sweep then costs the critical path of one column
// (its memory round trips and the instructions of its recurrences), not
// bandwidth. Here kStageWaves wavefronts share one segment of 64 columns:
// wavefront w loads layers w, w + kStageWaves, ... (all of its loads in one
// round trip), forms the right-hand sides s = f + sum_h T_h x_nb and writes
// s, the inverse pivots, the old iterate and the row's couplings Tr to LDS.
// After one block barrier the first two wavefronts solve the twisted
// factorisation of H_z in rolled loops over LDS (no per-layer address or
// branch arithmetic of a fully unrolled register solve), with the same
// recurrences as k_sweep: the forward values y_k overwrite s_k, the
// couplings Tr_next * ip_k overwrite the pivots.
constexpr int kStageWaves = 8;

// Dynamic LDS of k_smooth_staged (its static LDS holds NZ + 8 + 256 values).
template <typename T, int NZ, bool HAS_X>
constexpr size_t staged_lds_bytes() {
    return sizeof(T) * size_t(HAS_X ? 3 : 2) * NZ * 64;
}

template <typename T, int NZ, bool HAS_X>
__global__ __launch_bounds__(64 * kStageWaves) void k_smooth_staged(
    LevelView<T> L, const T* __restrict__ f, const T* __restrict__ xin, T* __restrict__ xout,
    T omega, int wpr) {
    extern __shared__ unsigned char smem_raw[];
    T* ls = reinterpret_cast<T*>(smem_raw);   // [NZ][64] s_k, then y_k
    T* lp = ls + NZ * 64;                      // [NZ][64] ip_k, then cb_k
    T* lx = lp + NZ * 64;                      // [NZ][64] old iterate (HAS_X)
    // separate LDS objects: the compiler then knows that the column loops'
    // stores to ls and lp leave the couplings alone
    __shared__ T ltr[NZ + 8];   // Tr_F of the row
    __shared__ T xch[256];      // the pair's exchange
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int lane = int(threadIdx.x & 63u);
    const Seg g = segment(int(blockIdx.x), L.nI, L.nJ, wpr);
    const NbB<T> b(g);
    const int nz = L.nz, nJ = L.nJ, J = g.J;
    const uint64_t Pb = uint64_t(L.plane) * sizeof(T);
    constexpr int Q = (NZ + kStageWaves - 1) / kStageWaves;
    {
        const int F = int(threadIdx.x);
        const T trF = F <= nz ? L.Tr[size_t(F) * size_t(nJ) + size_t(J)] : T(0);
        // the horizontal couplings of this wavefront's layers: lane q holds
        // those of layer wave + q kStageWaves (vector loads issued with the
        // stencil loads, read back with readlane)
        T ctl = T(0), cts = T(0), ctn = T(0);
        if (HAS_X && lane < Q) {
            const int kq = clampk(wave + lane * kStageWaves, nz);
            ctl = L.Tlam[size_t(kq) * size_t(nJ) + size_t(J)];
            cts = L.Tth[size_t(kq) * size_t(nJ + 1) + size_t(J)];
            ctn = L.Tth[size_t(kq) * size_t(nJ + 1) + size_t(J) + 1];
        }
        T rf[Q], rp[Q], rc[HAS_X ? Q : 1], rw[HAS_X ? Q : 1], re[HAS_X ? Q : 1],
            rs[HAS_X ? Q : 1], rn[HAS_X ? Q : 1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int kk = clampk(wave + q * kStageWaves, nz);
            rf[q] = ldb<T>(layer(f, kk, Pb), b.c);
            rp[q] = ldb<T>(layer(L.invp, kk, Pb), b.c);
            if constexpr (HAS_X) {
                gcptr xl = layer(xin, kk, Pb);
                rc[q] = ldb<T>(xl, b.c);
                rw[q] = ldb<T>(xl, b.w);
                re[q] = ldb<T>(xl, b.e);
                rs[q] = ldb<T>(xl, b.s);
                rn[q] = ldb<T>(xl, b.n);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (F <= nz) ltr[F] = trF;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = wave + q * kStageWaves;
            if (k < nz) {
                T s = rf[q];
                if constexpr (HAS_X) {
                    s += lane_value(ctl, q) * (rw[q] + re[q]) + lane_value(cts, q) * rs[q] +
                         lane_value(ctn, q) * rn[q];
                    lx[k * 64 + lane] = rc[q];
                }
                ls[k * 64 + lane] = s;
                lp[k * 64 + lane] = rp[q];
            }
        }
    }
    __syncthreads();
    if (wave >= 2) {
        __syncthreads();   // the solving pair's exchange barrier
        return;
    }
    const bool top = wave == 1;
    const int m = nz >> 1;
    const T keep = T(1) - omega;
    // forward: bottom eliminates layers 0..m-1 upward, top nz-1..m+1 downward
    T vp = T(0), sm = T(0), im = T(0);
    if (!top) {
#pragma unroll 4
        for (int k = 0; k < m; ++k) {
            const T s = ls[k * 64 + lane], ip = lp[k * 64 + lane];
            const T v = (s + ltr[k] * vp) * ip;
            ls[k * 64 + lane] = v;
            lp[k * 64 + lane] = ltr[k + 1] * ip;
            vp = v;
        }
        xch[lane] = vp;
    } else {
#pragma unroll 4
        for (int k = nz - 1; k > m; --k) {
            const T s = ls[k * 64 + lane], ip = lp[k * 64 + lane];
            const T v = (s + ltr[k + 1] * vp) * ip;
            ls[k * 64 + lane] = v;
            lp[k * 64 + lane] = ltr[k] * ip;
            vp = v;
        }
        sm = ls[m * 64 + lane];
        im = lp[m * 64 + lane];
        xch[64 + lane] = vp;
        xch[128 + lane] = sm;
        xch[192 + lane] = im;
    }
    __syncthreads();
    // meeting layer: x_m = (s_m + Tr_m y_{m-1} + Tr_{m+1} z_{m+1}) / d_m
    const T xm =
        (xch[128 + lane] + ltr[m] * xch[lane] + ltr[m + 1] * xch[64 + lane]) * xch[192 + lane];
    auto put = [&](int k, T z) {
        T out = omega * z;
        if constexpr (HAS_X) out += keep * lx[k * 64 + lane];
        if (g.valid) stb<T>(layer_w(xout, k, Pb), b.c, out);
    };
    T xv = xm;
    if (!top) {
#pragma unroll 4
        for (int k = m - 1; k >= 0; --k) {
            xv = ls[k * 64 + lane] + lp[k * 64 + lane] * xv;
            put(k, xv);
        }
    } else {
        put(m, xm);
#pragma unroll 4
        for (int k = m + 1; k < nz; ++k) {
            xv = ls[k * 64 + lane] + lp[k * 64 + lane] * xv;
            put(k, xv);
        }
    }
}

// The coarsest level in one launch from global memory: one block does every
// sweep from zero, segment by segment, ping-ponging between xa and xb, with
// a block barrier between sweeps (the global writes of a sweep are visible
// to the whole block after it). The result is in xa if sweeps is odd, else
// in xb.
template <typename T, int NZ, int D>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(LevelView<T> L, const T* __restrict__ f,
                                                       T* xa, T* xb, T omega, int sweeps,
                                                       int wpr) {
    __shared__ T xch[kBlock / 128][256];
    const PairOf p = pair_of_wave();
    const int nseg = L.nJ * wpr;
    for (int s = 0; s < sweeps; ++s) {
        T* xout = (s & 1) ? xb : xa;
        const T* xin = (s & 1) ? xa : xb;
        for (int s0 = 0; s0 < nseg; s0 += kBlock / 128) {
            const Seg g = segment(s0 + p.pair, L.nI, L.nJ, wpr);
            if (s == 0)
                sweep_segment<T, NZ, D, false>(L, f, nullptr, xout, omega, g, p.top,
                                               xch[p.pair]);
            else
                sweep_segment<T, NZ, D, true>(L, f, xin, xout, omega, g, p.top, xch[p.pair]);
            __syncthreads();
        }
    }
}

// The coarsest level in one launch with its data in LDS: a pair of
// wavefronts per 64 columns (plane <= kCoarseLdsColumns); the right-hand
// side, the pivots, the iterate and the coefficient tables are staged in
// LDS ([k][col]) once. A sweep reads the old neighbours from LDS, keeps its
// new half-column in registers, and after a block barrier overwrites the old
// iterate; a sweep then costs a few microseconds.
// UNIT: block b solves for the b-th unit vector instead of f and writes its
// result to row b of xout (rows of n values): the grid then computes the
// solve's explicit matrix, transposed, one row per block. The unit
// right-hand side is formed on the fly, not stored, and the horizontal
// coupling tables are read from global memory (L1 hits, fetched with the
// iterate one chunk ahead) instead of LDS: the smaller LDS footprint lets
// two blocks share a CU on the 4200-cell coarsest levels.
template <typename T, int NZ, bool UNIT>
__global__ __launch_bounds__(kBlock) void k_coarse_lds(LevelView<T> L, const T* __restrict__ f,
                                                       T* __restrict__ xout, T omega,
                                                       int sweeps) {
    extern __shared__ unsigned char smem_raw[];
    const int plane = int(L.plane), nz = L.nz, nJ = L.nJ, n = plane * nz;
    if constexpr (UNIT) xout += size_t(blockIdx.x) * size_t(n);
    T* sx = reinterpret_cast<T*>(smem_raw);
    T* sf = sx + n;                  // right-hand side (not UNIT)
    T* sp = sf + (UNIT ? 0 : n);
    T* stl = sp + n;                 // [nz][nJ] (not UNIT)
    T* sth = stl + (UNIT ? 0 : nz * nJ);        // [nz][nJ+1] (not UNIT)
    T* str = sth + (UNIT ? 0 : nz * (nJ + 1));  // [nz+1][nJ]
    T* xch = str + (nz + 1) * nJ;    // 256 per pair
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        sx[t] = T(0);   // the first sweep starts from zero: same code as the rest
        if constexpr (!UNIT) sf[t] = f[t];
        sp[t] = L.invp[t];
    }
    if constexpr (!UNIT) {
        for (int t = threadIdx.x; t < nz * nJ; t += blockDim.x) stl[t] = L.Tlam[t];
        for (int t = threadIdx.x; t < nz * (nJ + 1); t += blockDim.x) sth[t] = L.Tth[t];
    }
    for (int t = threadIdx.x; t < (nz + 1) * nJ; t += blockDim.x) str[t] = L.Tr[t];
    __syncthreads();
    const PairOf p = pair_of_wave();
    const int col = p.pair * 64 + int(threadIdx.x & 63u);
    const bool active = col < plane;
    const Nb b = neighbours<false>(active ? uint32_t(col) : 0u, L.nI, nJ);
    constexpr int D = ChunkDepth<T>::value;
    constexpr int NP = padded_steps<NZ, D>();
    const T keep = T(1) - omega;
    const int m = nz >> 1, nown = p.top ? nz - m : m;   // layers this wavefront writes
    T xk[NP];
    auto lay = [&](int t) {
        const int k = p.top ? nz - 1 - t : t;
        return k < 0 ? 0 : (k < nz ? k : nz - 1);
    };
    for (int s = 0; s < sweeps; ++s) {
        // opaque copies of the strides: the per-layer LDS addresses are then
        // recomputed each sweep instead of being hoisted out of the sweep
        // loop into hundreds of registers (the empty asm emits nothing)
        int pl = plane, nj = nJ;
        asm volatile("" : "+s"(pl), "+s"(nj));
        auto fetch = [&](int, int kk) {
            const T* xl = sx + kk * pl;
            CoarseRaw<T> r;
            if constexpr (UNIT) r.f = (kk * pl + int(b.c) == int(blockIdx.x)) ? T(1) : T(0);
            else r.f = sf[kk * pl + b.c];
            r.c = xl[b.c];
            r.w = xl[b.w];
            r.e = xl[b.e];
            r.s = xl[b.s];
            r.n = xl[b.n];
            const T* tl = UNIT ? L.Tlam : stl;
            const T* th = UNIT ? L.Tth : sth;
            r.tl = tl[kk * nj + b.J];
            r.ts = th[kk * (nj + 1) + b.J];
            r.tn = th[kk * (nj + 1) + b.J + 1];
            return r;
        };
        auto comb = [&](int t, int kk, const CoarseRaw<T>& r) -> T {
            xk[t] = r.c;
            return r.f + r.tl * (r.w + r.e) + r.ts * r.s + r.tn * r.n;
        };
        auto inv = [&](int kk) -> T { return sp[kk * pl + b.c]; };
        auto cpl = [&](int F) -> T { return str[F * nj + b.J]; };
        auto fsink = [](int, int, T) {};
        auto bload = [](int) -> T { return T(0); };
        auto sink = [&](int t, int, T z, T) { xk[t] = omega * z + keep * xk[t]; };
        twisted_column<T, NZ, D, false>(nz, p.top, xch + p.pair * 256, fetch, comb, inv, cpl,
                                        fsink, bload, sink);
        __syncthreads();   // every lane has read the old iterate
        if (active) {
#pragma unroll
            for (int t = 0; t < NP; ++t)
                if (t < nown) sx[lay(t) * plane + b.c] = xk[t];
        }
        __syncthreads();   // the new iterate is complete
    }
    if (active) {
#pragma unroll
        for (int t = 0; t < NP; ++t)
            if (t < nown) xout[size_t(lay(t)) * plane + b.c] = xk[t];
    }
}

}  // namespace

constexpr size_t kMaxLds = 160 * 1024;

// The staged sweep of a small level; false where the level is not small or
// the staging buffers do not fit in LDS.
template <typename T>
bool launch_staged(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega,
                   long long staged_columns, hipStream_t s) {
    if (L.plane >= staged_columns) return false;
    const int wpr = segments_per_row(L.nI);
    const int nb = L.nJ * wpr;
    bool launched = false;
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        auto go = [&](auto hx) {
            constexpr bool HX = decltype(hx)::value;
            constexpr size_t lds = staged_lds_bytes<T, NZ, HX>();
            if constexpr (lds + sizeof(T) * (NZ + 8 + 256) <= kMaxLds) {
                const void* fn =
                    reinterpret_cast<const void*>(&k_smooth_staged<T, NZ, HX>);
                if (lds > 64 * 1024 &&
                    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        int(lds)) != hipSuccess) {
                    (void)hipGetLastError();
                    return;
                }
                k_smooth_staged<T, NZ, HX>
                    <<<nb, 64 * kStageWaves, lds, s>>>(L, f, xin, xout, omega, wpr);
                launched = true;
            }
        };
        if (xin) go(std::true_type{});
        else go(std::false_type{});
    });
    return launched;
}

template <typename T>
void smooth(const LevelView<T>& L, const T* f, const T* xin, T* xout, T omega,
            long long staged_columns, hipStream_t s) {
    if (launch_staged<T>(L, f, xin, xout, omega, staged_columns, s)) return;
    sweep<T>(L, f, xin, xout, omega, s);
}

// Launch k_coarse_lds<T, NZ, UNIT> on `blocks` blocks; false if the level
// does not fit one block's LDS.
template <typename T, bool UNIT>
bool launch_coarse_lds(const LevelView<T>& L, const T* f, T* x, T omega, int sweeps,
                       size_t max_lds, int blocks, hipStream_t s) {
    const size_t lds = coarse_lds_bytes<T>(L.plane, L.nJ, L.nz, UNIT);
    if (L.plane > kCoarseLdsColumns || lds > max_lds) return false;
    const int threads = int((L.plane + 63) / 64) * 128;
    bool launched = false;
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_lds<T, NZ, UNIT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds)) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        k_coarse_lds<T, NZ, UNIT><<<blocks, threads, lds, s>>>(L, f, x, omega, sweeps);
        launched = true;
    });
    return launched;
}

template <typename T>
int coarse_solve(const LevelView<T>& L, const T* f, T* xa, T* xb, T omega, int sweeps,
                 size_t max_lds, hipStream_t s) {
    if (launch_coarse_lds<T, false>(L, f, xa, omega, sweeps, max_lds, 1, s)) return 0;
    const int wpr = segments_per_row(L.nI);
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
        k_coarse_solve<T, NZ, ChunkDepth<T>::value><<<1, kBlock, 0, s>>>(L, f, xa, xb, omega,
                                                                         sweeps, wpr);
    });
    return (sweeps & 1) ? 0 : 1;
}

bool coarse_basis(const LevelView<double>& L, double* Ct, double omega, int sweeps,
                  size_t max_lds, hipStream_t s) {
    const long long n = L.plane * L.nz;
    if (n > kDenseCoarseMax || n < 1) return false;
    return launch_coarse_lds<double, true>(L, nullptr, Ct, omega, sweeps, max_lds, int(n), s);
}

#define MG_INST(T)                                                                          \
    template void smooth<T>(const LevelView<T>&, const T*, const T*, T*, T, long long,      \
                            hipStream_t);                                                   \
    template int coarse_solve<T>(const LevelView<T>&, const T*, T*, T*, T, int, size_t,       \
                                 hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

}  // namespace mgk
