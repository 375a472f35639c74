// Context-free operator apply that allocates nothing: y = A x from the model k
// directly, for callers that cannot allocate device memory (code under graph
// capture, serving loops).  It runs the operator-apply kernel of
// hh_apply_operator; the one array that entry point keeps in its context,
// k^2 per node, lives here in a file-scope device array instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/hh.h"
#include "hh_common.h"
#include "hh_kernels.h"

namespace hh {
// error text of a failed call without a context (hh_last_error(NULL))
void set_error_without_context(const std::string& msg);
}  // namespace hh

using namespace hh;

namespace {

// k^2 of up to 2^23 nodes (64 MiB): the scratch of every call on a device.
// Each device that runs the library holds its own copy until the process ends.
constexpr long long NOALLOC_MAX_NODES = 1LL << 23;
__device__ __align__(256) double scratch[NOALLOC_MAX_NODES];

// Device address of `scratch` per device, looked up once per device with that
// device current (the array's name is a host-side stand-in, not an address).
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {};

hh_status fail(hh_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hh_status fail(hh_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    set_error_without_context(buf);
    return st;
}

}  // namespace

extern "C" hh_status hh_apply_operator_noalloc(const hh_config* cfg, const double* k, const void* x, void* y,
                                               int nrhs, void* hip_stream) {
    if (!cfg || !k || !x || !y) return fail(HH_ERR_ARG, "null argument");
    for (int d : {cfg->nx, cfg->ny, cfg->nz})
        if (d < 3 || d % 2 == 0) return fail(HH_ERR_ARG, "every axis needs an odd node count >= 3 (got %d)", d);
    if (!(cfg->h > 0.0) || !std::isfinite(cfg->h)) return fail(HH_ERR_ARG, "h must be > 0");
    if (cfg->bc != HH_BC_DIRICHLET && cfg->bc != HH_BC_SOMMERFELD) return fail(HH_ERR_ARG, "bad bc");
    if (nrhs < 1 || nrhs > 16) return fail(HH_ERR_ARG, "nrhs=%d outside 1..16", nrhs);
    Geo g;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.plane = cfg->nx * cfg->ny;
    g.n = (long long)cfg->nx * cfg->ny * cfg->nz;
    g.h = cfg->h;
    if (g.n > NOALLOC_MAX_NODES)
        return fail(HH_ERR_ARG, "a grid of %lld nodes exceeds the %lld nodes of the no-allocation scratch", g.n,
                    NOALLOC_MAX_NODES);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return fail(HH_ERR_HIP, "no usable current HIP device");
    double* k2 = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_scratch[dev]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(HH_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            g_scratch[dev] = static_cast<double*>(p);
        }
        k2 = g_scratch[dev];
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    // k^2 into the scratch (every entry the apply reads is written first), then
    // the operator apply of hh_apply_operator with the boundary wavenumber read
    // straight from k (the context keeps an exact copy of k for it)
    launch_level_k2<double>(s, g.n, k, k2);
    Launch L;
    L.block = 256;
    L.zb = std::min(4, g.nz);
    launch_apply<double>(s, cfg->bc, OP_PLAIN, g, L, nrhs, (const c128*)x, (c128*)y, k2, k, 1.0, 0.0, nullptr,
                         nullptr, 0, nullptr, GATE_ALL);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HH_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    return HH_OK;
}
