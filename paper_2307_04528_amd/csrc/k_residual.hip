// Operator apply, the FP64 refinement step (update + residual + norm), the
// deterministic reductions, and the setup / elementwise kernels.
//
// H is always evaluated in difference form (paper Section 2: Hu with H a
// Laplacian-like matrix):
//   (H x)_c = sum_faces T_f (x_c - x_nb) + M_c x_c.
#include "device.hpp"

namespace mgk {

constexpr int kResidualSync = 4;
// A k_residual_update block has one wavefront per row of its tile of R
// consecutive rows: R = 16 where that still gives at least
// kResidualTallBlocks blocks, else R = 4 (small levels would leave CUs
// idle). Every kResidualSync layers the block's wavefronts meet at a
// barrier: an XCD's L2 holds only a layer or two of all resident wavefronts'
// rows, so the latitude neighbours a wavefront reads are L2 hits only while
// the wavefronts that own those rows are at about the same layer. Measured
// on the 1024x768x70 shell: 2.03 -> 1.70 GB fetched and 470 -> 448 us per
// launch against 4-row tiles without the barrier.
constexpr int kResidualTallBlocks = 512;
constexpr int kResidualTallRows = 16;
// The walking refinement step: a range of layers per wavefront (the whole
// column of the 70-layer workloads; 16 layers on shallow levels), the
// layers whose loads are in flight ahead of the one being computed, and the
// same row tiles and barrier interval as above. Measured per launch on the
// 1024x768x70 shell (mixed solve): 446 us with whole columns against 458 us
// with two ranges of 35 layers; loads 2 or 4 layers ahead 467 and 468 us
// against 446; barriers every 8 layers or none 454 and 459 us; longitude
// neighbours loaded instead of shifted from the neighbour lanes 489 us.
// 16-row and 4-row tiles are within 1 % there; on 2560x1920x70 16-row
// tiles take 2.78-2.90 ms against 2.99-3.07 ms (FP64: 3.54-3.59 against
// 3.82-3.83 ms).
constexpr int kResidualRange = 70;
constexpr int kResidualShortRange = 16;
constexpr int kResidualAhead = 3;

static int residual_tile_rows(int nI, int nJ) {
    return dev::tiled_blocks(nJ, dev::segments_per_row(nI), kResidualTallRows) >=
                   kResidualTallBlocks
               ? kResidualTallRows
               : 4;
}

// Layers per walk: whole columns on levels with enough tall tiles to fill
// the GPU; ranges of kResidualShortRange layers on smaller levels, whose
// whole-column walks leave a few wavefronts per CU (384x192x70: 1152
// wavefronts, 54 us; in ranges of 16 layers five times as many, 45 us).
static int residual_walk_range(int nI, int nJ, int nz) {
    if (nz <= kResidualShortRange) return kResidualShortRange;
    return residual_tile_rows(nI, nJ) == kResidualTallRows ? kResidualRange
                                                           : kResidualShortRange;
}

namespace {
using namespace dev;

// Rows per block of the operator kernel (64 columns x this many rows: each
// wavefront one row) and layers per lane (a lane walks a chunk of layers of
// its column: the chunk's loads are in flight together, and the vertical
// neighbours come from the layers it already loaded).
constexpr int kApplyRows = 4;
// (FP32 2: adjoint solves on 1024x768x70 0.5-0.9 % slower with 4; FP64 4:
// 0.6 % slower with 2)
template <typename T>
constexpr int apply_layers() {
    return std::is_same<T, float>::value ? 2 : 4;
}

// y = H x (HAS_F = false) or y = f - H x, one lane per column and chunk of
// apply_layers layers, in blocks of 64 columns x kApplyRows rows (grid:
// column groups, row groups, layer chunks): a wavefront takes part of one
// row, so the row's couplings are wave-uniform and no lane divides its index.
template <typename T, bool HAS_F>
__global__ __launch_bounds__(64 * kApplyRows) void k_apply(LevelView<T> L,
                                                           const T* __restrict__ x,
                                                           const T* __restrict__ f,
                                                           T* __restrict__ y) {
    constexpr int NL = apply_layers<T>();
    const int nI = L.nI, nJ = L.nJ, nz = L.nz;
    const int i = int(blockIdx.x) * 64 + int(threadIdx.x);
    const int J = __builtin_amdgcn_readfirstlane(int(blockIdx.y) * kApplyRows +
                                                 int(threadIdx.y));
    const int k0 = int(blockIdx.z) * NL;
    if (i >= nI || J >= nJ) return;
    const size_t P = size_t(L.plane);
    const uint32_t c = uint32_t(J) * uint32_t(nI) + uint32_t(i);
    const uint32_t w = (i == 0) ? c + uint32_t(nI - 1) : c - 1u;
    const uint32_t e = (i == nI - 1) ? c - uint32_t(nI - 1) : c + 1u;
    const uint32_t sth = (J > 0) ? c - uint32_t(nI) : c;
    const uint32_t nth = (J < nJ - 1) ? c + uint32_t(nI) : c;
    auto clampk = [nz](int k) { return k < 0 ? 0 : (k < nz ? k : nz - 1); };
    // the column at layers k0-1 .. k0+NL (clamped: a boundary layer is its
    // own vertical neighbour, and its coupling term vanishes)
    T xv[NL + 2];
#pragma unroll
    for (int d = 0; d < NL + 2; ++d) xv[d] = x[size_t(clampk(k0 - 1 + d)) * P + c];
    T hs[NL];
#pragma unroll
    for (int d = 0; d < NL; ++d) {
        const int k = clampk(k0 + d);
        const T* xk = x + size_t(k) * P;
        const size_t t = size_t(k) * P + c;
        const T xc = xv[d + 1];
        const T xm = (k0 + d > 0) ? xv[d] : xc;
        const T xp = (k0 + d + 1 < nz) ? xv[d + 2] : xc;
        const T h = L.M[t] * xc +
                    hdiff(L.Tlam[k * nJ + J], L.Tth[k * (nJ + 1) + J],
                          L.Tth[k * (nJ + 1) + J + 1], xc, xk[w], xk[e], xk[sth], xk[nth]) +
                    L.Tr[k * nJ + J] * (xc - xm) + L.Tr[(k + 1) * nJ + J] * (xc - xp);
        hs[d] = HAS_F ? f[t] - h : h;
    }
#pragma unroll
    for (int d = 0; d < NL; ++d)
        if (k0 + d < nz) y[size_t(k0 + d) * P + c] = hs[d];
}

// Refinement step on the finest level, one lane per column (row-tiled
// segments, one wavefront per row of the block's tile), in the precision TU
// of the iterate (FP64; FP32 in the pure single-precision solve):
//   unew = uin + e (HAS_E; written to uout), r = b - H unew (stored as TR),
//   per-block partial sums of r^2 in FP64, and of b^2 when partials_b is set.
// Levels of more than 72 layers (the walking kernel below takes the others).
template <typename TU, typename TE, typename TR, int NZ, bool HAS_E, int R>
__global__ __launch_bounds__(64 * R) void k_residual_update(
    LevelView<TU> L, const TU* __restrict__ bv, const TU* __restrict__ uin,
    const TE* __restrict__ e, TU* __restrict__ uout, TR* __restrict__ r,
    double* __restrict__ partials, double* __restrict__ partials_b, int wpr) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const Seg g = tiled_segment(int(logical_block()), wave, R, L.nI, L.nJ, wpr);
    double acc = 0, accb = 0;
    {
        const Seg& nb = g;
        const NbB<TU> bu(nb);
        const NbB<TE> be(nb);
        const NbB<TR> br(nb);
        const int nJ = L.nJ, nz = L.nz;
        const uint64_t PU = uint64_t(L.plane) * sizeof(TU),
                       PE = uint64_t(L.plane) * sizeof(TE),
                       PR = uint64_t(L.plane) * sizeof(TR);
        // uin == nullptr: the iterate before the update is zero
        auto un = [&](int kk, uint32_t ou, uint32_t oe) -> TU {
            TU v = uin ? ldb<TU>(layer(uin, kk, PU), ou) : TU(0);
            if constexpr (HAS_E) v += TU(ldb<TE>(layer(e, kk, PE), oe));
            return v;
        };
        TU um = 0, uc = un(0, bu.c, be.c);
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
            const int kk = clampk(k, nz), kp = clampk(k + 1, nz);
            const TU up = un(kp, bu.c, be.c);
            const TU h =
                ldb<TU>(layer(L.M, kk, PU), bu.c) * uc +
                hdiff(tab(L.Tlam, kk * nJ + nb.J), tab(L.Tth, kk * (nJ + 1) + nb.J),
                      tab(L.Tth, kk * (nJ + 1) + nb.J + 1), uc, un(kk, bu.w, be.w),
                      un(kk, bu.e, be.e), un(kk, bu.s, be.s), un(kk, bu.n, be.n)) +
                tab(L.Tr, kk * nJ + nb.J) * (uc - um) + tab(L.Tr, (kk + 1) * nJ + nb.J) * (uc - up);
            const TU bk = ldb<TU>(layer(bv, kk, PU), bu.c);
            const TU rv = bk - h;
            if (k < nz && g.valid) {
                if constexpr (HAS_E) stb<TU>(layer_w(uout, kk, PU), bu.c, uc);
                stb<TR>(layer_w(r, kk, PR), br.c, TR(rv));
                acc += double(rv) * double(rv);
                accb += double(bk) * double(bk);
            }
            um = uc;
            uc = up;
            // keep the block's wavefronts within a few layers of each other
            if (k % kResidualSync == kResidualSync - 1) __syncthreads();
        }
    }
    if (partials_b) block_sum2_to(acc, accb, partials + blockIdx.x, partials_b + blockIdx.x);
    else block_sum_to(acc, partials + blockIdx.x);
}

// The same refinement step on levels whose step records cover every layer
// (nz <= kStepStride), walking ranges of LR layers: block b takes range
// b / tiles and the tile of R consecutive rows of one 64-column range
// b % tiles (one wavefront per row), and each wavefront walks its layers
// upward with the loads of the next P layers in flight, the layers below and
// above coming from the steps before and after. A row's couplings are its
// upward step record. FULLI: nI is a multiple of 64, so a lane's longitude
// neighbours are its neighbour lanes' values, and only lanes 0 and 63 load
// theirs. Every S layers the block's wavefronts meet at a barrier, so that
// the latitude neighbours they read are still in L2. HAS_U false: the
// iterate before the update is zero (the first update of a solve from
// u = 0), and uin is not read.
template <typename TU, typename TE, typename TR, bool HAS_E, bool HAS_U, int LR, int P, int R,
          int S, bool FULLI>
__global__ __launch_bounds__(64 * R) void k_residual_walk(
    LevelView<TU> L, const TU* __restrict__ bv, const TU* __restrict__ uin,
    const TE* __restrict__ e, TU* __restrict__ uout, TR* __restrict__ r,
    double* __restrict__ partials, double* __restrict__ partials_b, int wpr, int tiles) {
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int blk = int(logical_block());
    const int rg = blk / tiles;
    const Seg g = tiled_segment(blk - rg * tiles, wave, R, L.nI, L.nJ, wpr);
    const int nz = L.nz, kb = rg * LR;
    const uint32_t PU = uint32_t(L.plane) * sizeof(TU), PE = uint32_t(L.plane) * sizeof(TE),
                   PR = uint32_t(L.plane) * sizeof(TR);
    const rsrc_t ru = make_rsrc(HAS_U ? uin : bv, PU * uint32_t(nz)),
                 rb = make_rsrc(bv, PU * uint32_t(nz)),
                 rm = make_rsrc(L.M, PU * uint32_t(nz)),
                 re = make_rsrc(HAS_E ? (const void*)e : (const void*)uin, PE * uint32_t(nz)),
                 rw = make_rsrc(HAS_E ? (const void*)uout : (const void*)uin, PU * uint32_t(nz)),
                 rr = make_rsrc(r, PR * uint32_t(nz));
    const bool lane0 = (threadIdx.x & 63u) == 0;
    const uint32_t gcol = FULLI ? (lane0 ? g.w : g.e) : 0u;
    const uint32_t uc = g.c * sizeof(TU), us = g.s * sizeof(TU), un = g.n * sizeof(TU),
                   uw = (FULLI ? gcol : g.w) * sizeof(TU), ue = g.e * sizeof(TU);
    const uint32_t ec = g.c * sizeof(TE), es = g.s * sizeof(TE), en = g.n * sizeof(TE),
                   ew = (FULLI ? gcol : g.w) * sizeof(TE), ee = g.e * sizeof(TE);
    const uint32_t rc = g.c * sizeof(TR);
    const StepCoef<TU>* qp = L.sc + size_t(g.J) * kStepStride;

    // H is applied to a nonzero iterate (else r = b)
    constexpr bool HOP = HAS_U || HAS_E;
    // u + e at a cell of layer offsets (so_u, so_e); u = 0 without HAS_U
    auto un_at = [&](uint32_t ou, uint32_t oe, uint32_t so_u, uint32_t so_e) -> TU {
        TU v = TU(0);
        if constexpr (HAS_U) v = bld<TU>(ru, ou, so_u);
        if constexpr (HAS_E) v += TU(bld<TE>(re, oe, so_e));
        return v;
    };
    struct Lay {
        TU uc, us, un, uw, ue, b, m;
        TE ec, es, en, ew, ee;
        StepCoef<TU> q;
    };
    // the loads of step t (layer kb + t, clamped); only the column itself
    // for the layer above the range
    auto fetch = [&](int t, bool column_only) {
        Lay Q;
        if constexpr (!HAS_E) Q.ec = Q.es = Q.en = Q.ew = Q.ee = TE(0);
        if constexpr (!HAS_U) Q.uc = Q.us = Q.un = Q.uw = Q.ue = TU(0);
        const int k = clampk(kb + t, nz);
        const uint32_t su = uint32_t(k) * PU, se = uint32_t(k) * PE;
        if constexpr (HAS_U) Q.uc = bld<TU>(ru, uc, su);
        if constexpr (HAS_E) Q.ec = bld<TE>(re, ec, se);
        if (!column_only) {
            if constexpr (HAS_U) {
                Q.us = bld<TU>(ru, us, su);
                Q.un = bld<TU>(ru, un, su);
                Q.uw = bld<TU>(ru, uw, su);
                if constexpr (!FULLI) Q.ue = bld<TU>(ru, ue, su);
            }
            if constexpr (HAS_E) {
                Q.es = bld<TE>(re, es, se);
                Q.en = bld<TE>(re, en, se);
                Q.ew = bld<TE>(re, ew, se);
                if constexpr (!FULLI) Q.ee = bld<TE>(re, ee, se);
            }
            // b and the mass are read at the cell only: non-temporal loads
            Q.b = bld<TU, true>(rb, uc, su);
            if constexpr (HOP) {
                Q.m = bld<TU, true>(rm, uc, su);
                Q.q = step_rec(qp, size_t(k));
            }
        }
        return Q;
    };
    auto sum = [](TU u, TE x) -> TU {
        if constexpr (HAS_U && HAS_E) return u + TU(x);
        else if constexpr (HAS_E) return TU(x);
        else return u;
    };

    // the layer below the range, and its vertical coupling to the first
    // layer (0 at the bottom)
    const int kbm = kb > 0 ? kb - 1 : 0;
    const TU um0 = un_at(uc, ec, uint32_t(kbm) * PU, uint32_t(kbm) * PE);
    const TU tbm = step_rec(qp, size_t(kbm)).tc;
    TU um = um0, tb = kb > 0 ? tbm : TU(0);
    double acc = 0, accb = 0;
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
        const Lay& a = buf[(t + 1) % (P + 1)];
        const TU xc = sum(c.uc, c.ec), xp = sum(a.uc, a.ec);
        const TU xs = sum(c.us, c.es), xn = sum(c.un, c.en);
        TU xw, xe;
        if constexpr (FULLI) {
            const TU edge = sum(c.uw, c.ew);
            xw = from_below(edge, xc);
            xe = from_above(edge, xc);
        } else {
            xw = sum(c.uw, c.ew);
            xe = sum(c.ue, c.ee);
        }
        TU rv = c.b;
        if constexpr (HOP) {
            const StepCoef<TU> q = c.q;
            rv -= c.m * xc + hdiff(q.tl, q.ts, q.tn, xc, xw, xe, xs, xn) + tb * (xc - um) +
                  q.tc * (xc - xp);
            tb = q.tc;
        }
        // computed here, not sunk (with its loads) into the guarded stores
        asm volatile("" : "+v"(rv));
        const int k = kb + t;
        if (k < nz && g.valid) {
            if constexpr (HAS_E) bst(xc, rw, uc, uint32_t(k) * PU);
            bst(TR(rv), rr, rc, uint32_t(k) * PR);
            acc += double(rv) * double(rv);
            accb += double(c.b) * double(c.b);
        }
        um = xc;
        if (t % S == S - 1) __syncthreads();
    }
    if (partials_b) block_sum2_to(acc, accb, partials + blockIdx.x, partials_b + blockIdx.x);
    else block_sum_to(acc, partials + blockIdx.x);
}

// Block c sums the c-th array of partials (arrays `stride` apart) into out[c].
__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ p, int n,
                                                       long long stride,
                                                       double* __restrict__ out) {
    __shared__ double red[1024];
    p += blockIdx.x * stride;
    double acc = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) acc += p[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Setup: M = alpha V on the finest level; counts alpha values that are not
// finite and > 0.
__global__ __launch_bounds__(kBlock) void k_fine_mass(LevelView<double> L,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ alpha,
                                                      double* __restrict__ M, long long n,
                                                      double* __restrict__ partials) {
    double bad = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const int k = int(t / L.plane);
        const int J = int((t - k * L.plane) / L.nI);
        const double a = alpha[t];
        if (!(a > 0.0) || !isfinite(a)) bad += 1.0;
        if (M) M[t] = a * V[k * L.nJ + J];
    }
    block_sum_to(bad, partials + blockIdx.x);
}

// Setup: pivots of the twisted (two-sided) factorisation of H_z, per column.
// The column is eliminated from the bottom up to the layer below m = nz/2 and
// from the top down to the layer above it; layer m takes both. In row-sum
// form, with mt_k = M_k + 2 Tlam + Tth(south) + Tth(north) (the row sum of
// H_z at layer k) and Tr_F the coupling across face F (below layer F):
//   below m: g_0 = mt_0, g_k = mt_k + Tr_k g_{k-1} / (Tr_k + g_{k-1}),
//            stored 1 / (Tr_{k+1} + g_k)
//   above m: h_{nz-1} = mt_{nz-1}, h_k = mt_k + Tr_{k+1} h_{k+1} / (Tr_{k+1} + h_{k+1}),
//            stored 1 / (Tr_k + h_k)
//   at m:    stored 1 / (mt_m + Tr_m g_{m-1} / (Tr_m + g_{m-1})
//                            + Tr_{m+1} h_{m+1} / (Tr_{m+1} + h_{m+1}))
// These are the textbook pivots D_k - Tr^2 / p of each elimination without
// the cancellation (every g, h >= mt > 0).
__global__ __launch_bounds__(kBlock) void k_pivots(LevelView<double> L,
                                                   double* __restrict__ invp64,
                                                   float* __restrict__ invp32,
                                                   float* __restrict__ M32) {
    const uint32_t col = global_index();
    if (col >= uint32_t(L.plane)) return;
    const int J = int(col / uint32_t(L.nI)), nJ = L.nJ, nz = L.nz, m = nz / 2;
    auto off = [&](int k) { return size_t(k) * size_t(L.plane) + col; };
    auto mt = [&](int k) {
        return L.M[off(k)] + 2.0 * L.Tlam[k * nJ + J] + L.Tth[k * (nJ + 1) + J] +
               L.Tth[k * (nJ + 1) + J + 1];
    };
    auto tr = [&](int F) { return L.Tr[F * nJ + J]; };
    auto put = [&](int k, double ip) {
        invp64[off(k)] = ip;
        invp32[off(k)] = float(ip);
        M32[off(k)] = float(L.M[off(k)]);
    };
    double g = 0;
    for (int k = 0; k < m; ++k) {
        g = (k == 0) ? mt(0) : mt(k) + tr(k) * g / (tr(k) + g);
        put(k, 1.0 / (tr(k + 1) + g));
    }
    double h = 0;
    for (int k = nz - 1; k > m; --k) {
        h = (k == nz - 1) ? mt(k) : mt(k) + tr(k + 1) * h / (tr(k + 1) + h);
        put(k, 1.0 / (tr(k) + h));
    }
    double d = mt(m);
    if (m > 0) d += tr(m) * g / (tr(m) + g);
    if (m < nz - 1) d += tr(m + 1) * h / (tr(m + 1) + h);
    put(m, 1.0 / d);
}

__global__ __launch_bounds__(kBlock) void k_grad_alpha(LevelView<double> L,
                                                       const double* __restrict__ V,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ u,
                                                       double* __restrict__ g, uint32_t n) {
    const uint32_t t = global_index();
    if (t >= n) return;
    const uint32_t P = uint32_t(L.plane);
    const int k = int(t / P);
    const int J = int((t - uint32_t(k) * P) / uint32_t(L.nI));
    g[t] = -lam[t] * V[k * L.nJ + J] * u[t];
}

__global__ __launch_bounds__(kBlock) void k_cell_volumes(LevelView<double> L,
                                                         const double* __restrict__ V,
                                                         double* __restrict__ out, uint32_t n) {
    const uint32_t t = global_index();
    if (t >= n) return;
    const uint32_t P = uint32_t(L.plane);
    const int k = int(t / P);
    const int J = int((t - uint32_t(k) * P) / uint32_t(L.nI));
    out[t] = V[k * L.nJ + J];
}

template <typename TA, typename TB>
__global__ __launch_bounds__(kBlock) void k_cast(const TA* __restrict__ in, TB* __restrict__ out,
                                                 long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        out[t] = TB(in[t]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ out, T v, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        out[t] = v;
}

}  // namespace

template <typename T>
void apply(const LevelView<T>& L, const T* x, const T* f, T* y, hipStream_t s) {
    const dim3 grid(unsigned((L.nI + 63) / 64), unsigned((L.nJ + kApplyRows - 1) / kApplyRows),
                    unsigned((L.nz + apply_layers<T>() - 1) / apply_layers<T>()));
    if (f) k_apply<T, true><<<grid, dim3(64, kApplyRows), 0, s>>>(L, x, f, y);
    else k_apply<T, false><<<grid, dim3(64, kApplyRows), 0, s>>>(L, x, f, y);
}

template <typename TU, typename TE, typename TR>
int residual_update(const LevelView<TU>& L, const TU* b, const TU* uin, const TE* e, TU* uout,
                    TR* r, double* partials, double* partials_b, hipStream_t s) {
    const int wpr = segments_per_row(L.nI);
    const int nb = residual_update_blocks(L);
    const bool tall = residual_tile_rows(L.nI, L.nJ) == kResidualTallRows;
    if (L.nz <= kStepStride) {
        const int tiles = tiled_blocks(L.nJ, wpr, tall ? kResidualTallRows : 4);
        const bool full = L.nI % 64 == 0;
        auto go = [&](auto lrc, auto rc, auto fullc) {
            constexpr int LR = decltype(lrc)::value, R = decltype(rc)::value;
            constexpr bool FULLI = decltype(fullc)::value;
            constexpr int P = kResidualAhead, S = kResidualSync;
            if (e && uin)
                k_residual_walk<TU, TE, TR, true, true, LR, P, R, S, FULLI>
                    <<<nb, 64 * R, 0, s>>>(L, b, uin, e, uout, r, partials, partials_b, wpr, tiles);
            else if (e)
                k_residual_walk<TU, TE, TR, true, false, LR, P, R, S, FULLI>
                    <<<nb, 64 * R, 0, s>>>(L, b, uin, e, uout, r, partials, partials_b, wpr, tiles);
            else if (uin)
                k_residual_walk<TU, TE, TR, false, true, LR, P, R, S, FULLI>
                    <<<nb, 64 * R, 0, s>>>(L, b, uin, e, uout, r, partials, partials_b, wpr, tiles);
            else   // r = b: no neighbours (the same blocks and sums as with u = 0)
                k_residual_walk<TU, TE, TR, false, false, LR, P, R, S, false>
                    <<<nb, 64 * R, 0, s>>>(L, b, uin, e, uout, r, partials, partials_b, wpr, tiles);
        };
        auto by_rows = [&](auto lrc, auto fullc) {
            if (tall) go(lrc, std::integral_constant<int, kResidualTallRows>{}, fullc);
            else go(lrc, std::integral_constant<int, 4>{}, fullc);
        };
        auto by_full = [&](auto lrc) {
            if (full) by_rows(lrc, std::true_type{});
            else by_rows(lrc, std::false_type{});
        };
        if (residual_walk_range(L.nI, L.nJ, L.nz) == kResidualShortRange)
            by_full(std::integral_constant<int, kResidualShortRange>{});
        else
            by_full(std::integral_constant<int, kResidualRange>{});
        return nb;
    }
    with_nz(L.nz, [&](auto nzc) {
        constexpr int NZ = decltype(nzc)::value;
#define MG_RESIDUAL_LAUNCH(HE, R) \
    k_residual_update<TU, TE, TR, NZ, HE, R><<<nb, 64 * R, 0, s>>>(L, b, uin, e, uout, r, partials, \
                                                                  partials_b, wpr)
        if (tall) {
            if (e) MG_RESIDUAL_LAUNCH(true, kResidualTallRows);
            else MG_RESIDUAL_LAUNCH(false, kResidualTallRows);
        } else {
            if (e) MG_RESIDUAL_LAUNCH(true, 4); else MG_RESIDUAL_LAUNCH(false, 4);
        }
#undef MG_RESIDUAL_LAUNCH
    });
    return nb;
}

template <typename TU>
int residual_update_blocks(const LevelView<TU>& L) {
    const int tiles = tiled_blocks(L.nJ, segments_per_row(L.nI), residual_tile_rows(L.nI, L.nJ));
    if (L.nz > kStepStride) return tiles;
    const int lr = residual_walk_range(L.nI, L.nJ, L.nz);
    return tiles * ((L.nz + lr - 1) / lr);
}

void sum_partials(const double* partials, int n, double* out, hipStream_t s, int count,
                  long long stride) {
    k_sum_partials<<<count, 1024, 0, s>>>(partials, n, stride, out);
}

int fine_mass(const LevelView<double>& L, const double* V, const double* alpha, double* M,
              double* partials, hipStream_t s) {
    const long long n = L.plane * L.nz;
    const int nb = grid_stride_blocks(n);
    k_fine_mass<<<nb, kBlock, 0, s>>>(L, V, alpha, M, n, partials);
    return nb;
}

void pivots(const LevelView<double>& L, double* invp64, float* invp32, float* M32,
            hipStream_t s) {
    k_pivots<<<blocks_for(L.plane), kBlock, 0, s>>>(L, invp64, invp32, M32);
}

void grad_alpha(const LevelView<double>& L, const double* V, const double* lam,
                const double* u, double* g, hipStream_t s) {
    const long long n = L.plane * L.nz;
    k_grad_alpha<<<blocks_for(n), kBlock, 0, s>>>(L, V, lam, u, g, uint32_t(n));
}

void cell_volumes(const LevelView<double>& L, const double* V, double* out, hipStream_t s) {
    const long long n = L.plane * L.nz;
    k_cell_volumes<<<blocks_for(n), kBlock, 0, s>>>(L, V, out, uint32_t(n));
}

template <typename TA, typename TB>
void cast(const TA* in, TB* out, long long n, hipStream_t s) {
    k_cast<TA, TB><<<grid_stride_blocks(n), kBlock, 0, s>>>(in, out, n);
}

template <typename T>
void fill(T* out, T v, long long n, hipStream_t s) {
    k_fill<T><<<grid_stride_blocks(n), kBlock, 0, s>>>(out, v, n);
}

template void apply<float>(const LevelView<float>&, const float*, const float*, float*,
                           hipStream_t);
template void apply<double>(const LevelView<double>&, const double*, const double*, double*,
                            hipStream_t);
template int residual_update<double, float, float>(const LevelView<double>&, const double*,
                                                  const double*, const float*, double*,
                                                  float*, double*, double*, hipStream_t);
template int residual_update<double, double, double>(const LevelView<double>&,
                                                     const double*, const double*,
                                                     const double*, double*, double*,
                                                     double*, double*, hipStream_t);
template int residual_update<float, float, float>(const LevelView<float>&, const float*,
                                                 const float*, const float*, float*, float*,
                                                 double*, double*, hipStream_t);
template int residual_update_blocks<double>(const LevelView<double>&);
template int residual_update_blocks<float>(const LevelView<float>&);
template void cast<double, float>(const double*, float*, long long, hipStream_t);
template void cast<float, double>(const float*, double*, long long, hipStream_t);
template void cast<double, double>(const double*, double*, long long, hipStream_t);
template void fill<float>(float*, float, long long, hipStream_t);
template void fill<double>(double*, double, long long, hipStream_t);

}  // namespace mgk
