// Host build of the library's certified binary32 overlap tests -- the polygon
// separating-axis filter and the polyhedron XenoCollide walk (with the
// binary64 set-up it starts from) -- for CPU tests against the oracle.  Built
// with hipcc --offload-host-only; no GPU code runs.
#include <cmath>
#include <cstdint>

#include "../paper_1509_04692_amd/csrc/mpr32.hpp"
#include "../paper_1509_04692_amd/csrc/overlap32.hpp"
#include "../paper_1509_04692_amd/csrc/overlap64.hpp"

using namespace hpmc;

// verts: nv x 3 (row-major); r: n x 3; qa, qb: n x 4 (w, x, y, z).
// out[i] = 0 no overlap, 1 overlap, 2 uncertain.
extern "C" int mpr32_pairs(const double* verts, int nv, int64_t n, const double* r, const double* qa,
                           const double* qb, int32_t* out) {
    if (nv < 4 || nv > kMaxPolyhedronVerts) return -1;
    static SpeciesDev P;
    P = SpeciesDev{};
    P.nv = nv;
    double rmax = 0.0;
    for (int k = 0; k < nv; ++k) {
        P.vx[k] = verts[3 * k];
        P.vy[k] = verts[3 * k + 1];
        P.vz[k] = verts[3 * k + 2];
        const double rr = std::sqrt((P.vx[k] * P.vx[k] + P.vy[k] * P.vy[k]) + P.vz[k] * P.vz[k]);
        rmax = rr > rmax ? rr : rmax;
    }
    P.R = std::nextafter(rmax, INFINITY);
    const double tol = 1e-12 * (P.R + P.R);
    P.tol2 = tol * tol;
    fill_mpr32_tables(P, tol);
    for (int64_t i = 0; i < n; ++i) {
        const Minkowski64 mk = polyhedron_setup64(V3{r[3 * i], r[3 * i + 1], r[3 * i + 2]},
                                                  Quat{qa[4 * i], qa[4 * i + 1], qa[4 * i + 2], qa[4 * i + 3]},
                                                  Quat{qb[4 * i], qb[4 * i + 1], qb[4 * i + 2], qb[4 * i + 3]});
        const double t[3] = {mk.t.x, mk.t.y, mk.t.z};
        out[i] = polyhedron_overlap32(P, mk.M.m, t);
    }
    return 0;
}

// verts: nv x 2 (CCW); r: n x 2; za, zb: n x 2 (cos, sin).
// out[i] = 0 no overlap, 1 overlap, 2 uncertain.  margin_scale multiplies
// the certification margin (1 = the library's; tests shrink it to show that
// the comparison notices); symmetric selects the filter for polygons with
// the rotational symmetry of their vertex count (-3 if the shape lacks it).
extern "C" int sat32_pairs(const double* verts, int nv, int64_t n, const double* r, const double* za,
                           const double* zb, int32_t* out, double margin_scale, int symmetric) {
    if (nv < 3 || nv > kMaxPolyVerts) return -1;
    static SpeciesDev P;
    P = SpeciesDev{};
    P.nv = nv;
    double rmax = 0.0;
    for (int k = 0; k < nv; ++k) {
        P.vx[k] = verts[2 * k];
        P.vy[k] = verts[2 * k + 1];
        const double rr = std::sqrt(P.vx[k] * P.vx[k] + P.vy[k] * P.vy[k]);
        rmax = rr > rmax ? rr : rmax;
    }
    P.R = std::nextafter(rmax, INFINITY);
    if (!fill_polygon_tables(P)) return -2;
    P.sat_margin_scale = (float)(P.sat_margin_scale * margin_scale);
    P.sat_margin_regular = (float)(P.sat_margin_regular * margin_scale);
    if (symmetric && !P.regular) return -3;
    for (int64_t i = 0; i < n; ++i)
        out[i] = symmetric ? polygon_overlap32_regular<0>(P, r[2 * i], r[2 * i + 1], za[2 * i],
                                                          za[2 * i + 1], zb[2 * i], zb[2 * i + 1])
                           : polygon_overlap32<0>(P, r[2 * i], r[2 * i + 1], za[2 * i], za[2 * i + 1],
                                                  zb[2 * i], zb[2 * i + 1]);
    return 0;
}
