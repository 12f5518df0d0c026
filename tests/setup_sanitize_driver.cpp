// Host-side setup (the hierarchy planner behind mg_setup, mg_plan and
// mg_plan_tables) driven over many grids and options, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer. Every table and map of
// every level is read back and checked for the invariants the device code
// relies on; the process exits non-zero on a violated invariant, and the
// sanitizers abort it on an invalid access or undefined behaviour.
#include <cmath>
#include <cstdio>
#include <vector>

#include "setup.hpp"

namespace {

int failures = 0;

void expect(bool ok, const char* what, int nlon, int nlat, int nlev, int l) {
    if (!ok) {
        std::fprintf(stderr, "FAIL %s: grid %dx%dx%d level %d\n", what, nlon, nlat, nlev, l);
        ++failures;
    }
}

void check(int nlon, int nlat, int nlev, double stretch, int levels, double threshold) {
    mg_grid g{nlon, nlat, nlev, 1.0, 0.01, stretch, 1.0};
    mg_options o{};
    o.levels = levels;
    o.nu_pre = 2;
    o.nu_post = 2;
    o.coarse_sweeps = 40;
    o.max_iters = 100;
    o.omega = 0.8;
    o.semi_threshold = threshold;
    o.smooth_lo = 1.0 / 3.0;
    o.smooth_hi = 2.0;
    o.staged_columns = 65536;
    o.stall_factor = 0.9;
    o.stall_iters = 3;
    o.graphs = 1;
    if (!mgs::validate(g, o).empty()) {
        ++failures;
        std::fprintf(stderr, "FAIL validate rejected %dx%dx%d\n", nlon, nlat, nlev);
        return;
    }
    mgs::Hierarchy H;
    if (!mgs::plan(g, levels, threshold, H).empty() || H.levels.empty()) {
        ++failures;
        std::fprintf(stderr, "FAIL plan %dx%dx%d\n", nlon, nlat, nlev);
        return;
    }
    double total0 = 0;
    for (size_t l = 0; l < H.levels.size(); ++l) {
        const mgs::Level& L = H.levels[l];
        const int nI = L.nI, nJ = L.nJ, nz = L.nz, il = int(l);
        expect(nz == nlev, "layers", nlon, nlat, nlev, il);
        expect(int(L.V.size()) == nz * nJ && int(L.Tlam.size()) == nz * nJ &&
                   int(L.Tth.size()) == nz * (nJ + 1) && int(L.Tr.size()) == (nz + 1) * nJ,
               "table sizes", nlon, nlat, nlev, il);
        double total = 0;
        for (int k = 0; k < nz; ++k)
            for (int J = 0; J < nJ; ++J) {
                const double v = L.V[size_t(k) * nJ + J];
                expect(v > 0 && std::isfinite(v), "volume", nlon, nlat, nlev, il);
                expect(L.Tlam[size_t(k) * nJ + J] > 0, "Tlam", nlon, nlat, nlev, il);
                total += v * nI;
            }
        for (int k = 0; k < nz; ++k) {
            expect(L.Tth[size_t(k) * (nJ + 1)] == 0.0 &&
                       L.Tth[size_t(k) * (nJ + 1) + nJ] == 0.0,
                   "polar faces", nlon, nlat, nlev, il);
            for (int F = 1; F < nJ; ++F)
                expect(L.Tth[size_t(k) * (nJ + 1) + F] > 0, "Tth", nlon, nlat, nlev, il);
        }
        for (int J = 0; J < nJ; ++J) {
            expect(L.Tr[J] == 0.0 && L.Tr[size_t(nz) * nJ + J] == 0.0, "Neumann faces",
                   nlon, nlat, nlev, il);
            for (int F = 1; F < nz; ++F)
                expect(L.Tr[size_t(F) * nJ + J] > 0, "Tr", nlon, nlat, nlev, il);
        }
        if (l == 0) total0 = total;
        expect(std::fabs(total - total0) <= 1e-12 * total0, "total volume", nlon, nlat, nlev,
               il);
        if (l > 0) {
            const mgs::Level& Fi = H.levels[l - 1];
            expect(nI * 2 == Fi.nI, "halved longitudes", nlon, nlat, nlev, il);
            int next = 0;
            for (int J = 0; J < nJ; ++J) {
                const int f0 = L.child_first[J], c = L.child_count[J];
                expect(f0 == next && (c == 1 || c == 2), "child rows", nlon, nlat, nlev, il);
                next = f0 + c;
                for (int e = 0; e < 4; ++e) {
                    const int r = L.ptrow[4 * J + e];
                    expect(r >= -1 && r < Fi.nJ, "ptrow", nlon, nlat, nlev, il);
                }
            }
            expect(next == Fi.nJ, "rows covered", nlon, nlat, nlev, il);
            for (int j = 0; j < Fi.nJ; ++j) {
                expect(Fi.crow_of[j] >= 0 && Fi.crow_of[j] < nJ, "crow_of", nlon, nlat, nlev,
                       il);
                for (int s = 0; s < 2; ++s) {
                    const int r = Fi.prow[2 * j + s];
                    expect(r >= 0 && r < nJ && std::isfinite(Fi.pw[2 * j + s]), "prow",
                           nlon, nlat, nlev, il);
                }
            }
        }
    }
    for (int nu = 1; nu <= 4; ++nu)
        for (int k = 0; k < nu; ++k) {
            const double w = mgs::sweep_omega(o, nu, k);
            expect(w > 0 && w < 4 && std::isfinite(w), "sweep omega", nlon, nlat, nlev, -1);
        }
}

}  // namespace

int main() {
    const int lons[] = {2, 4, 6, 8, 12, 16, 34, 64, 96, 100, 128, 384};
    const int lats[] = {2, 4, 6, 8, 10, 32, 48, 50, 192};
    const int levs[] = {1, 2, 7, 16, 70, 128};
    int grids = 0;
    for (int nlon : lons)
        for (int nlat : lats)
            for (int nlev : levs)
                for (int levels : {0, 1, 4})
                    for (double t : {2.0, 4.0}) {
                        check(nlon, nlat, nlev, nlev > 64 ? 1.05 : 1.1, levels, t);
                        ++grids;
                    }
    check(1024, 768, 70, 1.07, 0, 2.0);
    check(1024, 768, 70, 1.07, 0, 4.0);
    std::printf("%d grids, %d failures\n", grids + 2, failures);
    return failures ? 1 : 0;
}
