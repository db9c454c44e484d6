// sc_timestep.hip -- the outer loop of the method on gfx950: the first-order
// Euler update of the configuration (section 3.2, Eq. time-step: centres by
// U, orientation quaternions by Psi(theta) Omega with Psi from the quaternion
// kinematics of section 2), the unit quaternion of a given axis, and the warm
// start of a step's LCP from the previous step's solution, matched pair by
// pair through the previous incidence lists (no sort).
#include <cmath>

#include "sc_common.hpp"
#include "sc_plan.hpp"

namespace sc {

namespace {

// Body axis e_z rotated by the unit quaternion (s, p):
// R e_z = (s^2 - p.p) e_z + 2 p_z p + 2 s (p x e_z).
__device__ __forceinline__ V3 quat_axis(double s, V3 p) {
    const double c = s * s - dot(p, p);
    return v3(2.0 * p.z * p.x + 2.0 * s * p.y, 2.0 * p.z * p.y - 2.0 * s * p.x,
              c + 2.0 * p.z * p.z);
}

// c += dt U, theta += dt Psi(theta) Omega (Psi = 1/2 [-p^T; s I - [p]x]),
// theta normalised, axis = R(theta) e_z.
__global__ void k_advance(int n, double *pos, double *quat, double *axis, const double *u_nc,
                          const double *u_c, double dt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double u[6];
    for (int a = 0; a < 6; ++a)
        u[a] = u_nc[6 * static_cast<long long>(k) + a] +
               (u_c ? u_c[6 * static_cast<long long>(k) + a] : 0.0);
    double *c = pos + 3 * static_cast<long long>(k);
    c[0] += dt * u[0];
    c[1] += dt * u[1];
    c[2] += dt * u[2];
    double *q = quat + 4 * static_cast<long long>(k);
    const double s = q[0];
    const V3 p = v3(q[1], q[2], q[3]), w = v3(u[3], u[4], u[5]);
    const V3 pw = cross(p, w);
    double ns = s - 0.5 * dt * dot(p, w);
    V3 np = p + (0.5 * dt) * (s * w - pw);
    const double inv = 1.0 / sqrt(ns * ns + dot(np, np));
    ns *= inv;
    np = inv * np;
    q[0] = ns;
    q[1] = np.x;
    q[2] = np.y;
    q[3] = np.z;
    store3(axis + 3 * static_cast<long long>(k), quat_axis(ns, np));
}

// The rotation taking e_z to the unit axis a along the shortest arc:
// normalise (1 + a_z, e_z x a); a = -e_z gives the half turn about x.
__global__ void k_quat_from_axis(int n, const double *axis, double *quat) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const V3 a = load3(axis + 3 * static_cast<long long>(k));
    double s = 1.0 + a.z;
    V3 p = v3(-a.y, a.x, 0.0);
    if (s < 1e-12) {
        s = 0.0;
        p = v3(1.0, 0.0, 0.0);
    }
    const double inv = 1.0 / sqrt(s * s + dot(p, p));
    double *q = quat + 4 * static_cast<long long>(k);
    q[0] = s * inv;
    q[1] = p.x * inv;
    q[2] = p.y * inv;
    q[3] = p.z * inv;
}

// gamma0_l of contact l = (i, j) of the current step: the previous step's
// gamma of the same pair, found among the previous contacts of i (its
// incidence list under its previous rank), else 0 (always 0 without a
// previous step).
__global__ void k_map_gamma(int nc, const int *ci, const int *cj, int have_prev, Plan prev,
                            const int *pci, const int *pcj, const double *pgamma,
                            double *gamma0) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    double v = 0.0;
    if (!have_prev) {
        gamma0[l] = v;
        return;
    }
    const int i = ci[l], j = cj[l];
    const int r = prev.rank[i];
    for (int e = prev.inc_ptr[r]; e < prev.inc_ptr[r + 1]; ++e) {
        const int m = prev.inc[e] >> 1;
        if (pci[m] == i && pcj[m] == j) {
            v = pgamma[m];
            break;
        }
    }
    gamma0[l] = v;
}

}  // namespace

}  // namespace sc

using namespace sc;

extern "C" int sc_advance(int32_t n, double *pos, double *quat, double *axis,
                          const double *u_nc, const double *u_c, double dt, void *stream) {
    if (n < 0 || !(dt > 0.0) || !std::isfinite(dt)) return SC_ERR_INVALID;
    if (n == 0) return SC_OK;
    if (!pos || !quat || !axis || !u_nc) return SC_ERR_INVALID;
    k_advance<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(n, pos, quat, axis,
                                                                           u_nc, u_c, dt);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

extern "C" int sc_quat_from_axis(int32_t n, const double *axis, double *quat, void *stream) {
    if (n < 0) return SC_ERR_INVALID;
    if (n == 0) return SC_OK;
    if (!axis || !quat) return SC_ERR_INVALID;
    k_quat_from_axis<<<grid_for(n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(n, axis, quat);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

extern "C" int sc_map_gamma(int32_t n, const sc_contacts *prev, const double *gamma_prev,
                            const sc_contacts *cur, double *gamma0, void *stream) {
    if (n < 0 || !prev || !cur || prev->count < 0 || prev->count > prev->capacity ||
        cur->count < 0 || cur->count > cur->capacity)
        return SC_ERR_INVALID;
    const int nc = cur->count;
    if (nc == 0) return SC_OK;
    if (!gamma0 || !cur->ci || !cur->cj) return SC_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int have = prev->count > 0 && n > 0;
    Plan pl{};
    if (have && (!gamma_prev || !prev->ci || !prev->cj ||
                 !carve_plan(prev->plan, prev->plan_bytes, n, prev->capacity, pl)))
        return SC_ERR_INVALID;
    k_map_gamma<<<grid_for(nc), kBlock, 0, s>>>(nc, cur->ci, cur->cj, have, pl, prev->ci,
                                                prev->cj, gamma_prev, gamma0);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}
