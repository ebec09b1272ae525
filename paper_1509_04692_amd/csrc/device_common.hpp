// Device arithmetic of the sweep whose binary64 results must be reproducible
// bit for bit: the counter-based random stream, uniform conversion, the
// small-angle sin/cos polynomial, cell coordinates, periodic wrap and minimum
// image.  Every expression is written in its pinned evaluation order; the
// library is compiled with -ffp-contract=off so none is fused.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies with hi/lo swaps, Weyl-sequence key schedule.  The counter is
// (sweep, purpose << 28 | select, id, replica) and the key the 64-bit seed,
// giving every trial move its own stream (the role of the hash-based
// generator of Sec. 2.5).
// ---------------------------------------------------------------------------
enum Purpose : uint32_t { kShift = 1u, kSelect = 2u, kMove = 3u };

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32x32 -> 64-bit multiply each (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint4 draw(uint32_t t, uint32_t purpose, uint32_t select, uint32_t id,
                                      uint32_t replica, uint32_t k0, uint32_t k1) {
    return philox4x32_10(make_uint4(t, (purpose << 28) | select, id, replica), k0, k1);
}

// (w + 1/2) 2^-32: exact in binary64, strictly inside (0, 1).
__device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// floor(w n / 2^32), an index in [0, n).
__device__ __forceinline__ uint32_t index_below(uint32_t w, uint32_t n) { return __umulhi(w, n); }

// ---------------------------------------------------------------------------
// sin and cos of a rotation angle |delta| <= a (small): Taylor polynomials
// through delta^15 and delta^16, evaluated by Horner's rule in delta^2 with
// the coefficients (-1)^k / k! rounded to binary64 (folded at compile time).
// ---------------------------------------------------------------------------
constexpr double inv_factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f = f * (double)i;
    return 1.0 / f;
}
constexpr double sin_coef(int k) { return (k % 2 == 1) ? -inv_factorial(2 * k + 1) : inv_factorial(2 * k + 1); }
constexpr double cos_coef(int k) { return (k % 2 == 1) ? -inv_factorial(2 * k) : inv_factorial(2 * k); }

__device__ __forceinline__ void small_angle_sincos(double delta, double& c, double& s) {
    constexpr double ks[8] = {sin_coef(0), sin_coef(1), sin_coef(2), sin_coef(3),
                              sin_coef(4), sin_coef(5), sin_coef(6), sin_coef(7)};
    constexpr double kc[9] = {cos_coef(0), cos_coef(1), cos_coef(2), cos_coef(3), cos_coef(4),
                              cos_coef(5), cos_coef(6), cos_coef(7), cos_coef(8)};
    const double x2 = delta * delta;
    double ps = ks[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) {
        ps = ps * x2;
        ps = ps + ks[k];
    }
    s = delta * ps;
    double pc = kc[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        pc = pc * x2;
        pc = pc + kc[k];
    }
    c = pc;
}

// ---------------------------------------------------------------------------
// Grid geometry (Sec. 2.2.1): coordinate in the frame of the grid shifted by
// s in (0, w) and the cell it falls in; periodic wrap of a coordinate
// displaced by less than L; minimum image of a separation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double grid_coord(double x, double s, double L) {
    const double y = x - s;
    return y < 0.0 ? y + L : y;
}

__device__ __forceinline__ int cell_of_coord(double y, double inv_w, int n) {
    int j = (int)(y * inv_w);
    j = j > n - 1 ? n - 1 : j;
    return j < 0 ? 0 : j;  // only reachable for positions outside [0, L)
}

__device__ __forceinline__ int cell_coord(double x, double s, double L, double inv_w, int n) {
    return cell_of_coord(grid_coord(x, s, L), inv_w, n);
}

__device__ __forceinline__ double wrap_periodic(double x, double L) {
    double y = x;
    if (x >= L)
        y = x - L;
    else if (x < 0.0)
        y = x + L;
    return y >= L ? 0.0 : y;
}

__device__ __forceinline__ double min_image(double r, double L, double inv_L) {
    return r - L * rint(r * inv_L);
}

// ---------------------------------------------------------------------------
// Quaternions: Hamilton product with each component summed left to right,
// and the rotation matrix of a unit quaternion.
// ---------------------------------------------------------------------------
struct Quat { double w, x, y, z; };

__host__ __device__ inline Quat qmul(const Quat& p, const Quat& q) {
    Quat o;
    o.w = ((p.w * q.w - p.x * q.x) - p.y * q.y) - p.z * q.z;
    o.x = ((p.w * q.x + p.x * q.w) + p.y * q.z) - p.z * q.y;
    o.y = ((p.w * q.y - p.x * q.z) + p.y * q.w) + p.z * q.x;
    o.z = ((p.w * q.z + p.x * q.y) - p.y * q.x) + p.z * q.w;
    return o;
}

struct Mat3 { double m[3][3]; };

__host__ __device__ inline Mat3 rotation_matrix(const Quat& q) {
    Mat3 r;
    r.m[0][0] = 1.0 - 2.0 * (q.y * q.y + q.z * q.z);
    r.m[0][1] = 2.0 * (q.x * q.y - q.w * q.z);
    r.m[0][2] = 2.0 * (q.x * q.z + q.w * q.y);
    r.m[1][0] = 2.0 * (q.x * q.y + q.w * q.z);
    r.m[1][1] = 1.0 - 2.0 * (q.x * q.x + q.z * q.z);
    r.m[1][2] = 2.0 * (q.y * q.z - q.w * q.x);
    r.m[2][0] = 2.0 * (q.x * q.z - q.w * q.y);
    r.m[2][1] = 2.0 * (q.y * q.z + q.w * q.x);
    r.m[2][2] = 1.0 - 2.0 * (q.x * q.x + q.y * q.y);
    return r;
}

// ---------------------------------------------------------------------------
// Wave64 helpers.
// ---------------------------------------------------------------------------
// Mask of the lanes where p holds (an SGPR pair, no VALU work).
__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of m below this lane (v_mbcnt_lo / v_mbcnt_hi).
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace hpmc
