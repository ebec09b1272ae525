// Host-only stand-in for the HIP runtime entry points that libhpmc's host
// code calls (test infrastructure).  Loaded with RTLD_GLOBAL before the
// library in a process without a GPU, it lets hpmc_init / hpmc_sweep /
// hpmc_autotune run their host logic: kernel launches and copies are checked
// and logged instead of executed.  Every pointer argument of a launch and
// every device side of a copy must lie inside a region the test registered
// (the caller's positions, orientations and workspace); device-to-host copies
// return zeros (no overlaps, valid state).
#include <cxxabi.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace {
struct dim3s {
    uint32_t x, y, z;
};
struct Region {
    uintptr_t base, size;
};
std::vector<Region> g_regions;
std::map<const void*, std::string> g_names;
std::map<const void*, size_t> g_var_size;
std::map<const void*, void*> g_var_mem;
dim3s g_grid{}, g_block{};
size_t g_shm = 0;
void* g_stream = nullptr;
long g_fake = 0x1000;
long g_launches = 0, g_violations = 0;
FILE* g_log = nullptr;

bool inside(uintptr_t p, uintptr_t n) {
    for (const Region& r : g_regions)
        if (p >= r.base && p + n <= r.base + r.size) return true;
    return false;
}
void violation(const char* what, const std::string& where) {
    ++g_violations;
    if (g_log) fprintf(g_log, "VIOLATION %s in %s\n", what, where.c_str());
}
std::string demangle(const std::string& m) {
    int st = 0;
    char* d = abi::__cxa_demangle(m.c_str(), nullptr, nullptr, &st);
    std::string r = (st == 0 && d) ? d : m;
    free(d);
    return r;
}
}  // namespace

extern "C" {
// -- test controls ---------------------------------------------------------
void stub_add_region(uintptr_t base, uintptr_t size);
void stub_add_region(uintptr_t base, uintptr_t size) { g_regions.push_back(Region{base, size}); }
void stub_open_log(const char* path) { g_log = fopen(path, "w"); }
long stub_launches() { return g_launches; }
long stub_violations() { return g_violations; }

// -- runtime entry points --------------------------------------------------
void** __hipRegisterFatBinary(const void*) {
    static void* h[4];
    return h;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* host_fun, char*, const char* device_name, unsigned int, void*,
                           void*, void*, void*, int*) {
    g_names[host_fun] = device_name;
}
// Device variables: a host buffer of the variable's size stands in for it
// once its address is asked for, and becomes a valid region.
void __hipRegisterVar(void**, char* host_var, char*, const char*, int, size_t size, int, int) {
    g_var_size[host_var] = size & 0xffffffffu;
}
int hipGetSymbolAddress(void** dev, const void* symbol) {
    const auto it = g_var_size.find(symbol);
    if (it == g_var_size.end()) return 1;
    void*& mem = g_var_mem[symbol];
    if (mem == nullptr) {
        mem = calloc(1, it->second);
        stub_add_region((uintptr_t)mem, it->second);
    }
    *dev = mem;
    return 0;
}
int __hipPushCallConfiguration(dim3s grid, dim3s block, size_t shm, void* stream) {
    g_grid = grid;
    g_block = block;
    g_shm = shm;
    g_stream = stream;
    return 0;
}
int __hipPopCallConfiguration(dim3s* grid, dim3s* block, size_t* shm, void** stream) {
    *grid = g_grid;
    *block = g_block;
    *shm = g_shm;
    *stream = g_stream;
    return 0;
}
constexpr size_t kLdsLimit = 160 * 1024;  // gfx950 LDS per work-group

int hipLaunchKernel(const void* f, dim3s grid, dim3s block, void** args, size_t shm, void*) {
    ++g_launches;
    const std::string name = demangle(g_names.count(f) ? g_names[f] : std::string("?"));
    if (g_log) fprintf(g_log, "launch %s grid(%u,%u,%u) block(%u,%u,%u)\n", name.c_str(), grid.x, grid.y,
                       grid.z, block.x, block.y, block.z);
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x == 0 || block.x > 1024) violation("launch shape", name);
    if (shm > kLdsLimit) violation("dynamic LDS", name);
    // the parameter list of the kernel's demangled signature: every pointer
    // argument must point into a registered region
    const size_t lp = name.find('('), rp = name.rfind(')');
    if (lp == std::string::npos || rp == std::string::npos || rp <= lp + 1) return 0;
    const std::string ps = name.substr(lp + 1, rp - lp - 1);
    int depth = 0, i = 0;
    std::string cur;
    auto check = [&](const std::string& t) {
        if (t.find('*') != std::string::npos) {
            uintptr_t v;
            memcpy(&v, args[i], sizeof v);
            if (!inside(v, 1)) violation("pointer argument", name + " #" + std::to_string(i));
        }
        ++i;
    };
    for (char c : ps) {
        if (c == '<' || c == '(') depth++;
        if (c == '>' || c == ')') depth--;
        if (c == ',' && depth == 0) {
            check(cur);
            cur.clear();
        } else {
            cur += c;
        }
    }
    if (!cur.empty()) check(cur);
    return 0;
}
int hipMemcpyAsync(void* dst, const void* src, size_t n, int kind, void*) {
    if (g_log) fprintf(g_log, "memcpy kind %d n %zu\n", kind, n);
    const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
    if ((kind == 1 || kind == 3) && !inside(d, n)) violation("copy destination", "hipMemcpyAsync");
    if ((kind == 2 || kind == 3) && !inside(s, n)) violation("copy source", "hipMemcpyAsync");
    if (kind == 2) memset(dst, 0, n);
    return 0;
}
int hipStreamSynchronize(void*) { return 0; }
int hipDeviceSynchronize() { return 0; }
int hipGetDevice(int* d) {
    *d = 0;
    return 0;
}
int hipDeviceGetAttribute(int* v, int, int) {
    *v = (int)kLdsLimit;
    return 0;
}
int hipFuncSetAttribute(const void* f, int, int value) {
    if (value < 0 || (size_t)value > kLdsLimit) violation("LDS limit", demangle(g_names[f]));
    return 0;
}
int hipGetLastError() { return 0; }
int hipEventCreate(void** e) {
    *e = (void*)(g_fake++);
    return 0;
}
int hipEventCreateWithFlags(void** e, unsigned) {
    *e = (void*)(g_fake++);
    return 0;
}
int hipEventDestroy(void*) { return 0; }
int hipEventElapsedTime(float* ms, void*, void*) {
    *ms = 1.0f;
    return 0;
}
int hipEventRecord(void*, void*) { return 0; }
int hipEventSynchronize(void*) { return 0; }
int hipStreamCreateWithFlags(void** s, unsigned) {
    *s = (void*)(g_fake++);
    return 0;
}
int hipStreamDestroy(void*) { return 0; }
int hipStreamWaitEvent(void*, void*, unsigned) { return 0; }
int hipStreamBeginCapture(void*, int) { return 0; }
int hipStreamEndCapture(void*, void** g) {
    *g = (void*)(g_fake++);
    return 0;
}
int hipGraphInstantiate(void** e, void*, void*, char*, size_t) {
    *e = (void*)(g_fake++);
    return 0;
}
int hipGraphDestroy(void*) { return 0; }
int hipGraphExecDestroy(void*) { return 0; }
int hipGraphLaunch(void*, void*) { return 0; }
}
