// Grid transfers of the horizontal-only hierarchy (paper Sections 2, 2.2):
//   restriction R: sum over the children (2 longitudes x 1 or 2 rows), fused
//                  with the residual f - H x (the paper restricts the residual);
//   prolongation P: cell-centred bilinear interpolation;
// and, for the transposed V-cycle, P^T and the transpose of the fused
// residual restriction.
#include "device.hpp"

namespace mgk {

// Coarse levels with more columns than this restrict with one lane per coarse
// column (registers reuse the vertical neighbours); smaller ones with one lane
// per coarse cell (no per-lane layer chain, latency hidden by parallelism).
#ifndef MG_RESTRICT_COLUMN_ABOVE
#define MG_RESTRICT_COLUMN_ABOVE (1LL << 17)
#endif

namespace {
using namespace dev;

// Residual of the two or four children of coarse cell (Ic, Jc) in layer k,
// summed. Children rows j0 and j1 = j0 + two (two = 0: one row, weight 0 on
// the duplicate). xm/xc/xp are layer bases for k-1, k, k+1 (clamped; the
// vertical coefficients are 0 at the bottom and top).
template <typename T, bool HAS_X>
__device__ __forceinline__ T restrict_cell(const LevelView<T>& F, const TransferView<T>& X,
                                           const T* f, const T* x, int k, int Jc, int Ic) {
    const int nI = F.nI, nJ = F.nJ, nz = F.nz;
    const size_t P = size_t(F.plane);
    const int j0 = X.child_first[Jc];
    const int two = X.child_count[Jc] - 1;
    const int j1 = j0 + two;
    const T w1 = T(two);
    const uint32_t i0 = 2 * Ic, i1 = i0 + 1;
    const uint32_t r0 = uint32_t(j0) * nI, r1 = uint32_t(j1) * nI;
    const T* fk = f + size_t(k) * P;
    T acc = fk[r0 + i0] + fk[r0 + i1] + w1 * (fk[r1 + i0] + fk[r1 + i1]);
    if constexpr (HAS_X) {
        const uint32_t iw = (i0 == 0) ? nI - 1 : i0 - 1;
        const uint32_t ie = (i1 == uint32_t(nI) - 1) ? 0 : i1 + 1;
        const uint32_t rs = (j0 > 0) ? r0 - nI : r0;
        const uint32_t rn = (j1 < nJ - 1) ? r1 + nI : r1;
        const T* xk = x + size_t(k) * P;
        const T* xm = x + size_t(k > 0 ? k - 1 : 0) * P;
        const T* xp = x + size_t(k + 1 < nz ? k + 1 : k) * P;
        const T* Mk = F.M + size_t(k) * P;
        const T c00 = xk[r0 + i0], c01 = xk[r0 + i1], c10 = xk[r1 + i0], c11 = xk[r1 + i1];
        const T tl0 = F.Tlam[k * nJ + j0], tl1 = F.Tlam[k * nJ + j1];
        const T ts0 = F.Tth[k * (nJ + 1) + j0], tn0 = F.Tth[k * (nJ + 1) + j0 + 1];
        const T ts1 = F.Tth[k * (nJ + 1) + j1], tn1 = F.Tth[k * (nJ + 1) + j1 + 1];
        const T tb0 = F.Tr[k * nJ + j0], tt0 = F.Tr[(k + 1) * nJ + j0];
        const T tb1 = F.Tr[k * nJ + j1], tt1 = F.Tr[(k + 1) * nJ + j1];
        // a merged row's other row is its latitude neighbour
        const T n00 = two ? c10 : xk[rn + i0], n01 = two ? c11 : xk[rn + i1];
        const T s10 = two ? c00 : xk[rs + i0], s11 = two ? c01 : xk[rs + i1];
        const T h0 = Mk[r0 + i0] * c00 +
                     hdiff(tl0, ts0, tn0, c00, xk[r0 + iw], c01, xk[rs + i0], n00) +
                     Mk[r0 + i1] * c01 +
                     hdiff(tl0, ts0, tn0, c01, c00, xk[r0 + ie], xk[rs + i1], n01) +
                     tb0 * ((c00 - xm[r0 + i0]) + (c01 - xm[r0 + i1])) +
                     tt0 * ((c00 - xp[r0 + i0]) + (c01 - xp[r0 + i1]));
        const T h1 = Mk[r1 + i0] * c10 +
                     hdiff(tl1, ts1, tn1, c10, xk[r1 + iw], c11, s10, xk[rn + i0]) +
                     Mk[r1 + i1] * c11 +
                     hdiff(tl1, ts1, tn1, c11, c10, xk[r1 + ie], s11, xk[rn + i1]) +
                     tb1 * ((c10 - xm[r1 + i0]) + (c11 - xm[r1 + i1])) +
                     tt1 * ((c10 - xp[r1 + i0]) + (c11 - xp[r1 + i1]));
        acc -= h0 + w1 * h1;
    }
    return acc;
}

// One lane per coarse cell.
template <typename T, bool HAS_X>
__global__ __launch_bounds__(kBlock) void k_restrict_flat(LevelView<T> F, TransferView<T> X,
                                                          const T* __restrict__ f,
                                                          const T* __restrict__ x,
                                                          T* __restrict__ fc, uint32_t nc) {
    const uint32_t t = global_index();
    if (t >= nc) return;
    const uint32_t Pc = uint32_t(X.nIc) * X.nJc;
    const int k = int(t / Pc);
    const uint32_t colc = t - uint32_t(k) * Pc;
    const int Jc = int(colc / uint32_t(X.nIc));
    const int Ic = int(colc) - Jc * X.nIc;
    fc[t] = restrict_cell<T, HAS_X>(F, X, f, x, k, Jc, Ic);
}

// One lane per coarse column, walking the layers (for large levels): the
// four children's values of the layers below, at and above k stay in
// registers, so each x value is loaded once per lane. ROWU: every wavefront
// lies inside one coarse row, so the children rows and the tables are
// wave-uniform.
template <typename T, int NZ, bool ROWU>
__global__ __launch_bounds__(kBlock) void k_restrict_column(LevelView<T> F, TransferView<T> X,
                                                            const T* __restrict__ f,
                                                            const T* __restrict__ x,
                                                            T* __restrict__ fc) {
    const uint32_t colc = global_index();
    const uint32_t Pc = uint32_t(X.nIc) * X.nJc;
    if (colc >= Pc) return;
    const int nI = F.nI, nJ = F.nJ, nz = F.nz;
    int Jc = int(colc / uint32_t(X.nIc));
    if constexpr (ROWU) Jc = __builtin_amdgcn_readfirstlane(Jc);
    const int Ic = int(colc) - Jc * X.nIc;
    const int j0 = X.child_first[Jc];
    const int two = X.child_count[Jc] - 1;  // 0 or 1
    const int j1 = j0 + two;
    const T w1 = T(two);
    const uint32_t i0 = 2 * uint32_t(Ic), i1 = i0 + 1;
    const uint32_t iw = (i0 == 0) ? uint32_t(nI - 1) : i0 - 1;
    const uint32_t ie = (i1 == uint32_t(nI - 1)) ? 0u : i1 + 1;
    const uint32_t r0 = uint32_t(j0) * nI, r1 = uint32_t(j1) * nI;
    const uint32_t rs = (j0 > 0) ? r0 - nI : r0, rn = (j1 < nJ - 1) ? r1 + nI : r1;
    constexpr uint32_t S = sizeof(T);
    const uint32_t o00 = (r0 + i0) * S, o01 = (r0 + i1) * S, o10 = (r1 + i0) * S,
                   o11 = (r1 + i1) * S;
    const uint32_t ow0 = (r0 + iw) * S, oe0 = (r0 + ie) * S, ow1 = (r1 + iw) * S,
                   oe1 = (r1 + ie) * S;
    const uint32_t os0 = (rs + i0) * S, os1 = (rs + i1) * S, on0 = (rn + i0) * S,
                   on1 = (rn + i1) * S;
    const uint64_t Pb = uint64_t(F.plane) * S, Pcb = uint64_t(Pc) * S;
    const uint32_t oc = colc * S;
    T m00 = 0, m01 = 0, m10 = 0, m11 = 0;
    gcptr x0 = layer(x, 0, Pb);
    T c00 = ldb<T>(x0, o00), c01 = ldb<T>(x0, o01), c10 = ldb<T>(x0, o10), c11 = ldb<T>(x0, o11);
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        const int kk = clampk(k, nz), kp = clampk(k + 1, nz);
        gcptr fk = layer(f, kk, Pb), Mk = layer(F.M, kk, Pb), xk = layer(x, kk, Pb),
              xp = layer(x, kp, Pb);
        const T p00 = ldb<T>(xp, o00), p01 = ldb<T>(xp, o01), p10 = ldb<T>(xp, o10),
                p11 = ldb<T>(xp, o11);
        const T tl0 = tab(F.Tlam, kk * nJ + j0), tl1 = tab(F.Tlam, kk * nJ + j1);
        const T ts0 = tab(F.Tth, kk * (nJ + 1) + j0), tn0 = tab(F.Tth, kk * (nJ + 1) + j0 + 1);
        const T ts1 = tab(F.Tth, kk * (nJ + 1) + j1), tn1 = tab(F.Tth, kk * (nJ + 1) + j1 + 1);
        const T tb0 = tab(F.Tr, kk * nJ + j0), tt0 = tab(F.Tr, (kk + 1) * nJ + j0);
        const T tb1 = tab(F.Tr, kk * nJ + j1), tt1 = tab(F.Tr, (kk + 1) * nJ + j1);
        // a merged row's other row is its latitude neighbour
        const T n00 = two ? c10 : ldb<T>(xk, on0), n01 = two ? c11 : ldb<T>(xk, on1);
        const T s10 = two ? c00 : ldb<T>(xk, os0), s11 = two ? c01 : ldb<T>(xk, os1);
        const T h0 = ldb<T>(Mk, o00) * c00 +
                     hdiff(tl0, ts0, tn0, c00, ldb<T>(xk, ow0), c01, ldb<T>(xk, os0), n00) +
                     ldb<T>(Mk, o01) * c01 +
                     hdiff(tl0, ts0, tn0, c01, c00, ldb<T>(xk, oe0), ldb<T>(xk, os1), n01) +
                     tb0 * ((c00 - m00) + (c01 - m01)) + tt0 * ((c00 - p00) + (c01 - p01));
        const T h1 = ldb<T>(Mk, o10) * c10 +
                     hdiff(tl1, ts1, tn1, c10, ldb<T>(xk, ow1), c11, s10, ldb<T>(xk, on0)) +
                     ldb<T>(Mk, o11) * c11 +
                     hdiff(tl1, ts1, tn1, c11, c10, ldb<T>(xk, oe1), s11, ldb<T>(xk, on1)) +
                     tb1 * ((c10 - m10) + (c11 - m11)) + tt1 * ((c10 - p10) + (c11 - p11));
        const T acc = ldb<T>(fk, o00) + ldb<T>(fk, o01) +
                      w1 * (ldb<T>(fk, o10) + ldb<T>(fk, o11)) - (h0 + w1 * h1);
        if (k < nz) stb<T>(layer_w(fc, kk, Pcb), oc, acc);
        m00 = c00; m01 = c01; m10 = c10; m11 = c11;
        c00 = p00; c01 = p01; c10 = p10; c11 = p11;
    }
}

// x += P xc, one lane per fine cell: bilinear interpolation (3/4, 1/4 in
// longitude; the row weights of the map in latitude).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelView<T> F, TransferView<T> X,
                                                        const T* __restrict__ xc,
                                                        T* __restrict__ x, uint32_t n) {
    const uint32_t t = global_index();
    if (t >= n) return;
    const uint32_t P = uint32_t(F.plane);
    const int k = int(t / P);
    const uint32_t col = t - uint32_t(k) * P;
    const int j = int(col / uint32_t(F.nI));
    const int i = int(col) - j * F.nI;
    const int nIc = X.nIc;
    const int J0 = X.prow[2 * j], J1 = X.prow[2 * j + 1];
    const T w0 = X.pw[2 * j], w1 = X.pw[2 * j + 1];
    const int I = i >> 1;
    const int In = (i & 1) ? (I + 1 == nIc ? 0 : I + 1) : (I == 0 ? nIc - 1 : I - 1);
    const T* lay = xc + size_t(k) * nIc * X.nJc;
    const T* c0 = lay + J0 * nIc;
    const T* c1 = lay + J1 * nIc;
    const T a = T(0.75), b = T(0.25);
    x[t] += w0 * (a * c0[I] + b * c0[In]) + w1 * (a * c1[I] + b * c1[In]);
}

// xc = P^T x, one lane per coarse cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_T(LevelView<T> F, TransferView<T> X,
                                                      const T* __restrict__ x,
                                                      T* __restrict__ xc, uint32_t nc) {
    const uint32_t t = global_index();
    if (t >= nc) return;
    const uint32_t Pc = uint32_t(X.nIc) * X.nJc;
    const int k = int(t / Pc);
    const uint32_t colc = t - uint32_t(k) * Pc;
    const int Jc = int(colc / uint32_t(X.nIc));
    const int Ic = int(colc) - Jc * X.nIc;
    const int nIf = F.nI;
    const int iE = 2 * Ic, iO = 2 * Ic + 1;
    const int iW = (iE == 0) ? nIf - 1 : iE - 1;
    const int iEE = (iO + 1 == nIf) ? 0 : iO + 1;
    const T a = T(0.75), b = T(0.25);
    T acc = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = X.ptrow[4 * Jc + e];
        const T w = X.ptw[4 * Jc + e];
        const T* r = x + size_t(k) * F.plane + size_t(row < 0 ? 0 : row) * nIf;
        acc += w * (a * (r[iE] + r[iO]) + b * (r[iW] + r[iEE]));
    }
    xc[t] = acc;
}

// fb += y, xb -= H y with y = R^T fcb (every child takes its coarse value),
// one lane per fine cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inject_residual_adj(LevelView<T> F,
                                                                TransferView<T> X,
                                                                const T* __restrict__ fcb,
                                                                T* __restrict__ xb,
                                                                T* __restrict__ fb, uint32_t n) {
    const uint32_t t = global_index();
    if (t >= n) return;
    const uint32_t P = uint32_t(F.plane);
    const int nI = F.nI, nJ = F.nJ, nz = F.nz, nIc = X.nIc;
    const int k = int(t / P);
    const uint32_t col = t - uint32_t(k) * P;
    const int j = int(col / uint32_t(nI));
    const int i = int(col) - j * nI;
    const size_t Pc = size_t(nIc) * X.nJc;
    const int iw = (i == 0) ? nI - 1 : i - 1, ie = (i == nI - 1) ? 0 : i + 1;
    const int oc = X.crow_of[j] * nIc;
    const int cc = oc + (i >> 1), cw = oc + (iw >> 1), ce = oc + (ie >> 1);
    const int cs = (j > 0) ? X.crow_of[j - 1] * nIc + (i >> 1) : cc;
    const int cn = (j < nJ - 1) ? X.crow_of[j + 1] * nIc + (i >> 1) : cc;
    const T* lay = fcb + size_t(k) * Pc;
    const T yc = lay[cc];
    const T ym = fcb[size_t(k > 0 ? k - 1 : 0) * Pc + cc];
    const T yp = fcb[size_t(k + 1 < nz ? k + 1 : k) * Pc + cc];
    const T h = F.M[t] * yc +
                hdiff(F.Tlam[k * nJ + j], F.Tth[k * (nJ + 1) + j], F.Tth[k * (nJ + 1) + j + 1],
                      yc, lay[cw], lay[ce], lay[cs], lay[cn]) +
                F.Tr[k * nJ + j] * (yc - ym) + F.Tr[(k + 1) * nJ + j] * (yc - yp);
    fb[t] += yc;
    xb[t] -= h;
}

}  // namespace

template <typename T>
void restrict_residual(const LevelView<T>& F, const TransferView<T>& X, const T* f,
                       const T* x, T* fc, hipStream_t s) {
    const long long Pc = (long long)X.nIc * X.nJc;
    if (x && Pc > MG_RESTRICT_COLUMN_ABOVE) {
        with_nz(F.nz, [&](auto nzc) {
            constexpr int NZ = decltype(nzc)::value;
            if (X.nIc % 64 == 0)
                k_restrict_column<T, NZ, true><<<blocks_for(Pc), kBlock, 0, s>>>(F, X, f, x, fc);
            else
                k_restrict_column<T, NZ, false><<<blocks_for(Pc), kBlock, 0, s>>>(F, X, f, x, fc);
        });
        return;
    }
    const long long nc = Pc * F.nz;
    if (x) k_restrict_flat<T, true><<<blocks_for(nc), kBlock, 0, s>>>(F, X, f, x, fc, uint32_t(nc));
    else k_restrict_flat<T, false><<<blocks_for(nc), kBlock, 0, s>>>(F, X, f, x, fc, uint32_t(nc));
}

template <typename T>
void prolong_add(const LevelView<T>& F, const TransferView<T>& X, const T* xc, T* x,
                 hipStream_t s) {
    const long long n = F.plane * F.nz;
    k_prolong_add<T><<<blocks_for(n), kBlock, 0, s>>>(F, X, xc, x, uint32_t(n));
}

template <typename T>
void prolong_transpose(const LevelView<T>& F, const TransferView<T>& X, const T* x, T* xc,
                       hipStream_t s) {
    const long long nc = (long long)X.nIc * X.nJc * F.nz;
    k_prolong_T<T><<<blocks_for(nc), kBlock, 0, s>>>(F, X, x, xc, uint32_t(nc));
}

template <typename T>
void inject_residual_adjoint(const LevelView<T>& F, const TransferView<T>& X, const T* fcb,
                             T* xb, T* fb, hipStream_t s) {
    const long long n = F.plane * F.nz;
    k_inject_residual_adj<T><<<blocks_for(n), kBlock, 0, s>>>(F, X, fcb, xb, fb, uint32_t(n));
}

#define MG_INST(T)                                                                       \
    template void restrict_residual<T>(const LevelView<T>&, const TransferView<T>&,      \
                                       const T*, const T*, T*, hipStream_t);              \
    template void prolong_add<T>(const LevelView<T>&, const TransferView<T>&, const T*,  \
                                 T*, hipStream_t);                                        \
    template void prolong_transpose<T>(const LevelView<T>&, const TransferView<T>&,      \
                                       const T*, T*, hipStream_t);                        \
    template void inject_residual_adjoint<T>(const LevelView<T>&, const TransferView<T>&, \
                                             const T*, T*, T*, hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

}  // namespace mgk
