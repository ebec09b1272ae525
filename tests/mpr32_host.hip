// Host build of the library's certified binary32 XenoCollide (and of the
// binary64 set-up it starts from), for CPU tests against the oracle.  Built
// with hipcc --offload-host-only; no GPU code runs.
#include <cmath>
#include <cstdint>

#include "../paper_1509_04692_amd/csrc/mpr32.hpp"
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
