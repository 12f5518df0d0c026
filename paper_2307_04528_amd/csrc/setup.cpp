// Host-side hierarchy construction. See setup.hpp.
//
// Geometry (paper Section 2: H is a Laplacian-like finite-volume operator;
// the discretisation itself is a reading, the paper gives none): a
// latitude-longitude shell with uniform longitudes, latitude rows given by
// their edges, and geometrically stretched layers counted from the surface.
//
// Coarsening (Sections 2.1-2.3): horizontal only; every level halves the
// longitudes; latitude rows merge in pairs only where both rows have
// anisotropy a = (dtheta / (cos(theta) dlambda))^2 <= threshold, pairing from
// the equator toward each pole (the northern hemisphere mirrors the
// southern one); coarse tables are rediscretised on the coarse geometry.
#include "setup.hpp"

#include <cmath>
#include <cstdio>

namespace mgs {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMinLongitudes = 4;

void vertical(const mg_grid& g, std::vector<double>& re, std::vector<double>& rc) {
    const int nz = g.nlev;
    re.assign(nz + 1, 0.0);
    rc.assign(nz, 0.0);
    re[0] = g.radius;
    double dz0 = (g.stretch == 1.0)
                     ? g.thickness / nz
                     : g.thickness * (g.stretch - 1.0) / (std::pow(g.stretch, nz) - 1.0);
    double dz = dz0;
    for (int k = 0; k < nz; ++k) {
        re[k + 1] = re[k] + dz;
        dz *= g.stretch;
    }
    for (int k = 0; k < nz; ++k) rc[k] = 0.5 * (re[k] + re[k + 1]);
}

// Fill the finite-volume tables of a level whose edges and nI are set.
void tables(const mg_grid& g, const std::vector<double>& re,
            const std::vector<double>& rc, Level& L) {
    const int nz = L.nz, nJ = L.nJ;
    const double K = g.K, dl = L.dlam;
    std::vector<double> th(nJ), dth(nJ), sdiff(nJ);
    for (int J = 0; J < nJ; ++J) {
        th[J] = 0.5 * (L.edges[J] + L.edges[J + 1]);
        dth[J] = L.edges[J + 1] - L.edges[J];
        sdiff[J] = std::sin(L.edges[J + 1]) - std::sin(L.edges[J]);
    }
    L.V.assign(size_t(nz) * nJ, 0.0);
    L.Tlam.assign(size_t(nz) * nJ, 0.0);
    L.Tth.assign(size_t(nz) * (nJ + 1), 0.0);
    L.Tr.assign(size_t(nz + 1) * nJ, 0.0);
    for (int k = 0; k < nz; ++k) {
        const double lo = re[k], hi = re[k + 1];
        const double shell_vol = (hi * hi * hi - lo * lo * lo) / 3.0;  // int r^2 dr
        const double shell_area = (hi * hi - lo * lo) / 2.0;          // int r dr
        for (int J = 0; J < nJ; ++J) {
            L.V[size_t(k) * nJ + J] = shell_vol * dl * sdiff[J];
            L.Tlam[size_t(k) * nJ + J] =
                K * shell_area * dth[J] / (rc[k] * std::cos(th[J]) * dl);
        }
        // interior latitude faces; the polar faces (F = 0, nJ) stay 0
        for (int F = 1; F < nJ; ++F) {
            L.Tth[size_t(k) * (nJ + 1) + F] =
                K * shell_area * std::cos(L.edges[F]) * dl / (rc[k] * (th[F] - th[F - 1]));
        }
    }
    // interior vertical faces; bottom (F = 0) and top (F = nz) stay 0
    for (int F = 1; F < nz; ++F) {
        const double r2 = re[F] * re[F];
        for (int J = 0; J < nJ; ++J)
            L.Tr[size_t(F) * nJ + J] = K * r2 * dl * sdiff[J] / (rc[F] - rc[F - 1]);
    }
    double amax = 0;
    for (int J = 0; J < nJ; ++J) {
        double t = dth[J] / (std::cos(th[J]) * dl);
        amax = std::fmax(amax, t * t);
    }
    L.max_anisotropy = amax;
}

double row_anisotropy(const Level& L, int J) {
    const double th = 0.5 * (L.edges[J] + L.edges[J + 1]);
    const double t = (L.edges[J + 1] - L.edges[J]) / (std::cos(th) * L.dlam);
    return t * t;
}

// Pair rows of the southern hemisphere from the equator toward the pole,
// mirror to the north. Returns, south to north, (first row, count) groups.
void group_rows(const Level& L, double threshold, std::vector<int>& first,
                std::vector<int>& count) {
    const int half = L.nJ / 2;
    std::vector<int> sf, sc;   // equator -> pole order
    int J = half - 1;
    while (J >= 0) {
        if (J >= 1 && row_anisotropy(L, J) <= threshold &&
            row_anisotropy(L, J - 1) <= threshold) {
            sf.push_back(J - 1);
            sc.push_back(2);
            J -= 2;
        } else {
            sf.push_back(J);
            sc.push_back(1);
            J -= 1;
        }
    }
    first.clear();
    count.clear();
    for (int g = int(sf.size()) - 1; g >= 0; --g) {  // south pole -> equator
        first.push_back(sf[g]);
        count.push_back(sc[g]);
    }
    for (size_t g = 0; g < sf.size(); ++g) {         // equator -> north pole
        const int last = sf[g] + sc[g] - 1;
        first.push_back(L.nJ - 1 - last);
        count.push_back(sc[g]);
    }
}

// Prolongation maps between fine level f and coarse level c.
void transfer_maps(Level& f, Level& c) {
    const int nJf = f.nJ, nJc = c.nJ;
    f.crow_of.assign(nJf, -1);
    for (int J = 0; J < nJc; ++J)
        for (int s = 0; s < c.child_count[J]; ++s) f.crow_of[c.child_first[J] + s] = J;
    auto centre = [](const Level& L, int J) { return 0.5 * (L.edges[J] + L.edges[J + 1]); };
    f.prow.assign(2 * nJf, 0);
    f.pw.assign(2 * nJf, 0.0);
    for (int j = 0; j < nJf; ++j) {
        const int J = f.crow_of[j];
        int J1 = J;
        double w0 = 1.0, w1 = 0.0;
        if (c.child_count[J] == 2) {
            // linear in theta toward the neighbouring coarse row on this side
            const double tf = centre(f, j), tc = centre(c, J);
            const int nb = (tf < tc) ? J - 1 : J + 1;
            if (nb >= 0 && nb < nJc) {
                const double tn = centre(c, nb);
                w0 = (tf - tn) / (tc - tn);
                w1 = 1.0 - w0;
                J1 = nb;
            }
        }
        f.prow[2 * j] = J;
        f.prow[2 * j + 1] = J1;
        f.pw[2 * j] = w0;
        f.pw[2 * j + 1] = w1;
    }
    // gather lists of the transpose: every (fine row, weight) pointing at J
    c.ptrow.assign(4 * nJc, -1);
    c.ptw.assign(4 * nJc, 0.0);
    std::vector<int> used(nJc, 0);
    for (int j = 0; j < nJf; ++j)
        for (int s = 0; s < 2; ++s) {
            const double w = f.pw[2 * j + s];
            if (w == 0.0) continue;
            const int J = f.prow[2 * j + s];
            const int e = used[J]++;
            c.ptrow[4 * J + e] = j;   // at most 4 rows reach any coarse row
            c.ptw[4 * J + e] = w;
        }
}

}  // namespace

std::string validate(const mg_grid& g, const mg_options& o) {
    char buf[256];
    if (g.nlon < 2 || g.nlon % 2 != 0) {
        std::snprintf(buf, sizeof buf, "nlon must be even and >= 2 (got %d)", g.nlon);
        return buf;
    }
    if (g.nlat < 2 || g.nlat % 2 != 0) {
        std::snprintf(buf, sizeof buf, "nlat must be even and >= 2 (got %d)", g.nlat);
        return buf;
    }
    if (g.nlev < 1 || g.nlev > MG_MAX_NLEV) {
        std::snprintf(buf, sizeof buf, "nlev must be in 1..%d (got %d)", MG_MAX_NLEV, g.nlev);
        return buf;
    }
    if (!(g.radius > 0) || !(g.thickness > 0) || !(g.stretch > 0) || !(g.K > 0) ||
        !std::isfinite(g.radius) || !std::isfinite(g.thickness) ||
        !std::isfinite(g.stretch) || !std::isfinite(g.K))
        return "radius, thickness, stretch and K must be finite and > 0";
    if (double(g.nlon) * g.nlat * g.nlev >= 536870912.0)
        return "grid too large (2^29 cells or more: an FP64 field must stay below 4 GiB)";
    if (o.levels < 0 || o.levels > MG_MAX_LEVELS) return "levels must be in 0..32";
    if (o.nu_pre < 1 || o.nu_post < 0 || o.nu_pre > 16 || o.nu_post > 16)
        return "need 1 <= nu_pre <= 16 and 0 <= nu_post <= 16";
    if (o.coarse_sweeps < 1 || o.coarse_sweeps > 1000) return "coarse_sweeps must be in 1..1000";
    if (o.max_iters < 0 || o.max_iters > MG_HIST - 1) return "max_iters must be in 0..127";
    if (!(o.omega > 0 && o.omega < 2)) return "omega must be in (0, 2)";
    if (!(o.stall_factor > 0) || !std::isfinite(o.stall_factor) || o.stall_iters < 0)
        return "stall_factor must be finite and > 0, stall_iters >= 0";
    if (o.graphs != 0 && o.graphs != 1) return "graphs must be 0 or 1";
    if (o.zero_guess != 0 && o.zero_guess != 1) return "zero_guess must be 0 or 1";
    if (o.poison != 0 && o.poison != 1) return "poison must be 0 or 1";
    if (!(o.semi_threshold > 0) || !std::isfinite(o.semi_threshold))
        return "semi_threshold must be finite and > 0";
    if (o.precision != MG_PREC_MIXED && o.precision != MG_PREC_FP64 &&
        o.precision != MG_PREC_FP32)
        return "precision must be MG_PREC_MIXED, MG_PREC_FP64 or MG_PREC_FP32";
    if (o.smooth_lo != 0.0 &&
        !(o.smooth_lo > 0 && o.smooth_hi > o.smooth_lo && std::isfinite(o.smooth_hi)))
        return "smoothing interval must be 0 or 0 < smooth_lo < smooth_hi";
    if (o.staged_columns < 0) return "staged_columns must be >= 0";
    if (o.profile < 0 || o.profile > 3) return "profile must be 0, 1, 2 or 3";
    return "";
}

double sweep_omega(const mg_options& o, int nu, int k) {
    if (o.smooth_lo == 0.0 || nu < 2) return o.omega;   // one sweep: omega
    // the k-th Chebyshev node of [lo, hi] (decreasing in k)
    const double lo = o.smooth_lo, hi = o.smooth_hi, pi = 3.14159265358979323846;
    const double lam = 0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos(pi * (2 * k + 1) / (2.0 * nu));
    return 1.0 / lam;
}

std::string plan(const mg_grid& g, int levels, double threshold, Hierarchy& H) {
    H.levels.clear();
    vertical(g, H.r_edge, H.r_centre);
    Level L0;
    L0.nI = g.nlon;
    L0.nJ = g.nlat;
    L0.nz = g.nlev;
    L0.dlam = 2.0 * kPi / g.nlon;
    L0.edges.resize(g.nlat + 1);
    for (int j = 0; j <= g.nlat; ++j) L0.edges[j] = -0.5 * kPi + j * (kPi / g.nlat);
    L0.edges[g.nlat] = 0.5 * kPi;
    tables(g, H.r_edge, H.r_centre, L0);
    H.levels.push_back(std::move(L0));
    while (int(H.levels.size()) < MG_MAX_LEVELS) {
        Level& cur = H.levels.back();
        if (levels > 0 && int(H.levels.size()) >= levels) break;
        if (levels == 0 && cur.max_anisotropy <= threshold) break;
        // halve the longitudes only while the count is even, and never below
        // kMinLongitudes cells around a circle (wider cells make the
        // cell-centred fluxes meaningless and the coarse correction harmful)
        if (cur.nI % 2 != 0 || cur.nI / 2 < kMinLongitudes) break;
        Level c;
        group_rows(cur, threshold, c.child_first, c.child_count);
        c.nI = cur.nI / 2;
        c.nJ = int(c.child_first.size());
        c.nz = cur.nz;
        c.dlam = 2.0 * kPi / c.nI;
        c.edges.push_back(cur.edges[0]);
        for (int J = 0; J < c.nJ; ++J)
            c.edges.push_back(cur.edges[c.child_first[J] + c.child_count[J]]);
        tables(g, H.r_edge, H.r_centre, c);
        transfer_maps(cur, c);
        H.levels.push_back(std::move(c));
    }
    return "";
}

}  // namespace mgs
