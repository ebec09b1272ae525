// Device arithmetic probe for the tests: runs the library's own device
// helpers (Philox4x32-10, the small-angle sin/cos polynomial, the minimum
// image) and the binary64 square root, division and rint that the sweep
// relies on, over arrays given by the host.  Test infrastructure only.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../paper_1509_04692_amd/csrc/device_common.hpp"

using namespace hpmc;

namespace {

__global__ void k_philox(const uint4* __restrict__ ctr, int64_t n, uint32_t k0, uint32_t k1,
                         uint4* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

__global__ void k_f64(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                      double* __restrict__ sq, double* __restrict__ dv, double* __restrict__ ri) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sq[i] = sqrt(a[i]);
    dv[i] = a[i] / b[i];
    ri[i] = rint(b[i]);
}

__global__ void k_sincos(const double* __restrict__ d, int64_t n, double* __restrict__ c,
                         double* __restrict__ s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double cc, ss;
    small_angle_sincos(d[i], cc, ss);
    c[i] = cc;
    s[i] = ss;
}

template <class T>
int to_device(const T* h, int64_t n, T** d) {
    if (hipMalloc((void**)d, sizeof(T) * (size_t)(n > 0 ? n : 1)) != hipSuccess) return -1;
    if (n > 0 && hipMemcpy(*d, h, sizeof(T) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) return -1;
    return 0;
}

template <class T>
int to_host(const T* d, int64_t n, T* h) {
    return (n > 0 && hipMemcpy(h, d, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) ? -1 : 0;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

// out[4i .. 4i+3] = Philox4x32-10(ctr[4i .. 4i+3], key (k0, k1)); host arrays.
int probe_philox(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t* out) {
    uint4 *dc = nullptr, *dout = nullptr;
    int rc = to_device(reinterpret_cast<const uint4*>(ctr), n, &dc);
    if (!rc && hipMalloc((void**)&dout, sizeof(uint4) * (size_t)(n > 0 ? n : 1)) != hipSuccess) rc = -1;
    if (!rc && n > 0) {
        k_philox<<<blocks(n), 256>>>(dc, n, k0, k1, dout);
        rc = hipDeviceSynchronize() == hipSuccess ? 0 : -1;
    }
    if (!rc) rc = to_host(dout, n, reinterpret_cast<uint4*>(out));
    (void)hipFree(dc);
    (void)hipFree(dout);
    return rc;
}

// sqrt(a), a / b and rint(b) elementwise; host arrays.
int probe_f64(const double* a, const double* b, int64_t n, double* sq, double* dv, double* ri) {
    double *da = nullptr, *db = nullptr, *ds = nullptr, *dd = nullptr, *dr = nullptr;
    int rc = to_device(a, n, &da);
    if (!rc) rc = to_device(b, n, &db);
    const size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    if (!rc && (hipMalloc((void**)&ds, bytes) != hipSuccess || hipMalloc((void**)&dd, bytes) != hipSuccess ||
                hipMalloc((void**)&dr, bytes) != hipSuccess))
        rc = -1;
    if (!rc && n > 0) {
        k_f64<<<blocks(n), 256>>>(da, db, n, ds, dd, dr);
        rc = hipDeviceSynchronize() == hipSuccess ? 0 : -1;
    }
    if (!rc) rc = to_host(ds, n, sq);
    if (!rc) rc = to_host(dd, n, dv);
    if (!rc) rc = to_host(dr, n, ri);
    for (double* p : {da, db, ds, dd, dr}) (void)hipFree(p);
    return rc;
}

// The sweep's cos/sin of small rotation angles; host arrays.
int probe_sincos(const double* d, int64_t n, double* c, double* s) {
    double *dd = nullptr, *dc = nullptr, *ds = nullptr;
    int rc = to_device(d, n, &dd);
    const size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    if (!rc && (hipMalloc((void**)&dc, bytes) != hipSuccess || hipMalloc((void**)&ds, bytes) != hipSuccess))
        rc = -1;
    if (!rc && n > 0) {
        k_sincos<<<blocks(n), 256>>>(dd, n, dc, ds);
        rc = hipDeviceSynchronize() == hipSuccess ? 0 : -1;
    }
    if (!rc) rc = to_host(dc, n, c);
    if (!rc) rc = to_host(ds, n, s);
    for (double* p : {dd, dc, ds}) (void)hipFree(p);
    return rc;
}

}  // extern "C"
