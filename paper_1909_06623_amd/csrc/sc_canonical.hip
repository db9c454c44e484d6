// sc_canonical.hip -- the permutation from the library's solver order of the
// contacts to the canonical order of the close-pair set: by ci, then cj (one
// constraint per pair i < j, section 3.1; a wall contact's cj = -1 - face is
// negative, so a particle's wall contacts come first).
//
// Every contact is on the incidence list of the plan's rank of its ci, so
// one thread per particle i finds the contacts that name it as ci there:
// their number is scanned into the canonical offset of i, and a contact's
// place among them is the number of those with a smaller cj. No sort and no
// atomics: the result depends only on the contact list.
#include "sc_common.hpp"
#include "sc_plan.hpp"

namespace {

__global__ void k_canon_count(int n, const int32_t *rank, const int32_t *inc_ptr,
                              const int32_t *inc, const int32_t *ci, int32_t *cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = rank[i];
    int c = 0;
    for (int e = inc_ptr[r]; e < inc_ptr[r + 1]; ++e) c += ci[inc[e] >> 1] == i;
    cnt[i] = c;
}

__global__ void k_canon_fill(int n, const int32_t *rank, const int32_t *inc_ptr,
                             const int32_t *inc, const int32_t *ci, const int32_t *cj,
                             const int32_t *off, int32_t *perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = rank[i], e0 = inc_ptr[r], e1 = inc_ptr[r + 1];
    for (int e = e0; e < e1; ++e) {
        const int l = inc[e] >> 1;
        if (ci[l] != i) continue;
        const int j = cj[l];
        int before = 0;
        for (int f = e0; f < e1; ++f) {
            const int m = inc[f] >> 1;
            before += (ci[m] == i) & (cj[m] < j);
        }
        perm[off[i] + before] = l;
    }
}

}  // namespace

extern "C" int sc_canonical_order(int32_t n, const sc_contacts *c, int32_t *perm, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (!c || n < 0 || c->count < 0 || c->count > c->capacity) return SC_ERR_INVALID;
    sc::Plan pl;
    if (!sc::carve_plan(c->plan, c->plan_bytes, n, c->capacity, pl)) return SC_ERR_INVALID;
    if (c->count == 0 || n == 0) return SC_OK;
    if (!perm || !c->ci || !c->cj) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < sc_workspace_bytes(n, c->capacity, SC_WS_BUILD))
        return SC_ERR_WORKSPACE;
    sc::Carver cv{static_cast<char *>(ws), ws_bytes};
    int32_t *cnt = cv.take<int32_t>(static_cast<size_t>(n) + 1);
    int32_t *tmp = cv.take<int32_t>(static_cast<size_t>(sc::scan_tmp_ints(n + 1)));
    if (!cv.ok) return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int b = sc::grid_for(n);
    k_canon_count<<<b, sc::kBlock, 0, s>>>(n, pl.rank, pl.inc_ptr, pl.inc, c->ci, cnt);
    sc::scan_exclusive(cnt, cnt, n, tmp, s);
    k_canon_fill<<<b, sc::kBlock, 0, s>>>(n, pl.rank, pl.inc_ptr, pl.inc, c->ci, c->cj, cnt,
                                         perm);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}
