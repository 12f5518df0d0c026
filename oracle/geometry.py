"""Shell geometry and the finite-volume transmissibilities of one grid level.

Test infrastructure (see the package docstring).

The paper (Section 2) only says H is a sparse, Laplacian-like matrix coming from
a Schur complement; it gives no discretisation. The reading taken here is the
cell-centred 7-point finite-volume form of -div(K grad u) + alpha u on a
latitude-longitude spherical shell, integrated over each cell:

  (Hu)_c = sum over faces f of c of T_f (u_c - u_nb(f)) + M_c u_c,

with exact-integral face areas and volumes and centre-to-centre distances.

Grid (longitude fastest; array index order [k][j][i]):
  * longitude: nlon cells of width dlam = 2 pi / nlon, periodic;
  * latitude: rows given by their edges, from -pi/2 (south pole) to +pi/2;
    a row's centre is the midpoint of its edges;
  * vertical: layer depths dz_k = dz_0 q^k counted upward from the surface,
    dz_0 = D (q-1)/(q^nz - 1) (D/nz if q = 1); r_{-1/2} = R, r_{k+1/2} =
    r_{k-1/2} + dz_k, r_k the midpoint.

Tables at one level (all i-independent because K is a constant):
  V[k,J]    = (r_{k+1/2}^3 - r_{k-1/2}^3)/3 * dlam * (sin th_{J+1/2} - sin th_{J-1/2})
  Tlam[k,J] = K * (r_{k+1/2}^2 - r_{k-1/2}^2)/2 * dth_J / (r_k cos th_J dlam)
  Tth[k,F]  = K * (r_{k+1/2}^2 - r_{k-1/2}^2)/2 * cos(e_F) * dlam / (r_k (th_F - th_{F-1}))
              for interior faces F = 1..nJ-1 (face F lies between rows F-1, F);
              0 at the two polar faces F = 0 and F = nJ (no flux across a pole)
  Tr[F,J]   = K * r_F^2 * dlam * s_J / (r_F - r_{F-1}) for interior vertical
              faces F = 1..nz-1 (between layers F-1 and F, at radius r_{F-1/2});
              0 at the bottom and top (homogeneous Neumann).
"""
from __future__ import annotations

import numpy as np


def vertical_coords(nz: int, radius: float, thickness: float, stretch: float):
    """Return (r_edge[nz+1], r_centre[nz]) of the geometrically stretched layers."""
    q = float(stretch)
    if q == 1.0:
        dz = np.full(nz, thickness / nz)
    else:
        dz0 = thickness * (q - 1.0) / (q ** nz - 1.0)
        dz = dz0 * q ** np.arange(nz, dtype=np.float64)
    r_edge = np.empty(nz + 1)
    r_edge[0] = radius
    for k in range(nz):
        r_edge[k + 1] = r_edge[k] + dz[k]
    r_centre = 0.5 * (r_edge[:-1] + r_edge[1:])
    return r_edge, r_centre


def fine_lat_edges(nlat: int) -> np.ndarray:
    """Uniform latitude edges -pi/2 + j pi/nlat, j = 0..nlat."""
    return -0.5 * np.pi + np.arange(nlat + 1, dtype=np.float64) * (np.pi / nlat)


class Level:
    """One grid level: sizes, latitude rows and FV tables.

    Attributes
      nlon, nlat, nz : cells per direction (nlat = number of latitude rows)
      edges          : latitude edges of the rows, length nlat+1
      dlam           : longitude width of a cell
      V, Tlam        : (nz, nlat) tables
      Tth            : (nz, nlat+1) latitude-face table
      Tr             : (nz+1, nlat) vertical-face table
      M              : (nz, nlat, nlon) mass term sum(alpha V) of the cell
      child_first, child_count : for a coarse level, the rows of the next
                       finer level that each row J aggregates
    """

    def __init__(self, nlon, edges, r_edge, r_centre, K):
        self.nlon = int(nlon)
        self.edges = np.asarray(edges, dtype=np.float64)
        self.nlat = len(self.edges) - 1
        self.nz = len(r_centre)
        self.dlam = 2.0 * np.pi / self.nlon
        self.K = float(K)
        self.r_edge = r_edge
        self.r_centre = r_centre
        self.child_first = None
        self.child_count = None
        self.M = None
        self._pivots = None
        self._build_tables()

    # --- geometry -----------------------------------------------------
    @property
    def theta(self):
        """Row centres: midpoints of the row edges."""
        return 0.5 * (self.edges[:-1] + self.edges[1:])

    @property
    def dtheta(self):
        return np.diff(self.edges)

    @property
    def sin_diff(self):
        return np.sin(self.edges[1:]) - np.sin(self.edges[:-1])

    def _build_tables(self):
        K, dlam = self.K, self.dlam
        re, rc = self.r_edge, self.r_centre
        nz, nJ = self.nz, self.nlat
        th, dth, sdiff = self.theta, self.dtheta, self.sin_diff

        vol_r = (re[1:] ** 3 - re[:-1] ** 3) / 3.0      # integral of r^2 dr
        area_r = (re[1:] ** 2 - re[:-1] ** 2) / 2.0      # integral of r dr

        self.V = vol_r[:, None] * dlam * sdiff[None, :]

        self.Tlam = K * area_r[:, None] * dth[None, :] / (
            rc[:, None] * np.cos(th)[None, :] * dlam)

        cos_face = np.cos(self.edges)
        cos_face[0] = 0.0          # the poles: no flux
        cos_face[-1] = 0.0
        Tth = np.zeros((nz, nJ + 1))
        if nJ > 1:
            dist = th[1:] - th[:-1]
            Tth[:, 1:nJ] = K * area_r[:, None] * cos_face[None, 1:nJ] * dlam / (
                rc[:, None] * dist[None, :])
        self.Tth = Tth

        Tr = np.zeros((nz + 1, nJ))
        if nz > 1:
            Tr[1:nz, :] = K * (re[1:nz] ** 2)[:, None] * dlam * sdiff[None, :] / (
                (rc[1:] - rc[:-1])[:, None])
        self.Tr = Tr

    @property
    def shape(self):
        return (self.nz, self.nlat, self.nlon)
