// Host-side setup of the multigrid hierarchy: shell geometry, finite-volume
// tables, the conditional semi-coarsening map and the transfer maps.
// Plain C++ (no HIP), FP64 throughout.
#pragma once

#include <string>
#include <vector>

#include "mg.h"

namespace mgs {

// One level of the hierarchy.
//
// Finite-volume tables (i-independent because K is a constant), with the
// exact-integral areas and volumes and centre-to-centre distances:
//   V[k*nJ+J]        cell volume
//   Tlam[k*nJ+J]     transmissibility of each longitude face of row J
//   Tth[k*(nJ+1)+F]  latitude face F (south of row F); 0 at the two poles
//   Tr[F*nJ+J]       vertical face F (below layer F); 0 at bottom and top
//
// Maps to the next coarser level (empty on the coarsest level):
//   crow_of[j]          coarse row of fine row j
//   prow[2j+s], pw[2j+s] latitude rows and weights used by prolongation
// Maps from the next finer level (empty on the finest level):
//   child_first[J], child_count[J]  fine rows aggregated by coarse row J
//   ptrow[4J+e], ptw[4J+e]          fine rows (or -1) and weights gathered by
//                                   the transpose of prolongation
struct Level {
    int nI = 0, nJ = 0, nz = 0;
    double dlam = 0;
    std::vector<double> edges;        // nJ+1 latitude edges
    std::vector<double> V, Tlam, Tth, Tr;
    std::vector<int> crow_of, prow;
    std::vector<double> pw;
    std::vector<int> child_first, child_count, ptrow;
    std::vector<double> ptw;
    double max_anisotropy = 0;
};

struct Hierarchy {
    std::vector<double> r_edge, r_centre;
    std::vector<Level> levels;
};

// Validate grid and options; returns an empty string or an error message.
std::string validate(const mg_grid& g, const mg_options& o);

// omega of sweep k (0-based) of a smoothing step of nu sweeps: o.omega, or
// 1/lambda_k for the Chebyshev nodes lambda_k of [smooth_lo, smooth_hi].
double sweep_omega(const mg_options& o, int nu, int k);

// Build the hierarchy (tables and maps) for the grid with the given level
// rule (levels == 0: automatic) and anisotropy threshold.
std::string plan(const mg_grid& g, int levels, double threshold, Hierarchy& out);

}  // namespace mgs
