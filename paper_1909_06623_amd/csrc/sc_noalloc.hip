// sc_noalloc.hip -- sc_solve_lcp for callers that cannot allocate device
// memory: the solve's workspace is a library-owned device array instead of
// a caller buffer.
//
// `scratch` is a file-scope device array; every GPU that loads the library
// holds its own copy until the process ends. In host code its name is only
// a host-side stand-in, so the device address is looked up once per device
// with hipGetSymbolAddress (with that device current) and only that address
// is ever handed to kernels or runtime calls.
#include <mutex>

#include "sc_common.hpp"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[SC_NOALLOC_SCRATCH_BYTES];

std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's `scratch`, looked up on first use.
int scratch_ptr(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SC_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SC_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SC_OK;
}

}  // namespace

extern "C" int sc_solve_lcp_noalloc(const sc_particles *p, const sc_contacts *c,
                                    const sc_solve_opts *opts, double *gamma, double *g,
                                    double *f_c, double *u_c, sc_stats *st, void *stream) {
    if (!p || !c || p->n < 0 || c->capacity < 0) return SC_ERR_INVALID;
    if (sc::solve_ws_bytes(p->n, c->capacity) > SC_NOALLOC_SCRATCH_BYTES) return SC_ERR_WORKSPACE;
    // every argument is checked before the first HIP call (the symbol lookup)
    const int bad = sc::check_solve_args(p, c, opts, gamma, g, st);
    if (bad) return bad;
    void *ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc != SC_OK) return rc;
    return sc::solve_lcp_on(p, c, opts, gamma, g, f_c, u_c, st, ws, SC_NOALLOC_SCRATCH_BYTES,
                            stream, false);
}
