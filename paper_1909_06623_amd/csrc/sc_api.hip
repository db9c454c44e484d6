// sc_api.hip -- library-level entry points: workspace sizing, error text,
// release of per-thread host resources, version.
#include "sc_common.hpp"

extern "C" size_t sc_workspace_bytes(int32_t n, int32_t capacity, int32_t what) {
    if (n < 0 || capacity < 0) return 0;
    const size_t a = sc::contacts_ws_bytes(n, capacity);
    const size_t b = sc::solve_ws_bytes(n, capacity);
    const size_t c = sc::adjoint_ws_bytes(n, capacity);
    switch (what) {
    case SC_WS_ALL: {
        const size_t m = a > b ? a : b;
        return m > c ? m : c;
    }
    case SC_WS_BUILD: return a;
    case SC_WS_SOLVE: return b;
    case SC_WS_ADJOINT: return c;
    default: return 0;
    }
}

extern "C" const char *sc_strerror(int code) {
    switch (code) {
    case SC_OK: return "ok";
    case SC_NOT_CONVERGED: return "not converged within max_iter (outputs hold the last iterate)";
    case SC_ERR_INVALID: return "invalid argument";
    case SC_ERR_CAPACITY: return "contact capacity too small (count holds the required rows)";
    case SC_ERR_NONFINITE: return "non-finite value in an input or an iterate";
    case SC_ERR_BOX: return "periodic box side below twice the interaction range";
    case SC_ERR_HIP: return "HIP runtime error";
    case SC_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
    case SC_ERR_TIMEOUT: return "a grid barrier of a persistent kernel timed out";
    default: return "unknown status code";
    }
}

extern "C" int sc_release(void) {
    if (hipDeviceSynchronize() != hipSuccess) return SC_ERR_HIP;
    sc::release_solve_host();
    sc::release_mob_host();
    return SC_OK;
}

extern "C" int sc_version(void) { return 370; }
