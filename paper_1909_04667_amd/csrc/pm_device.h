// Device code of the mesh interpolation (Sec. 3.3: four-point finite
// difference of the potential and CIC interpolation), shared by the
// single-system kernels (pm.hip) and the resident serving loop (server.hip).
#pragma once

#include "tpm_internal.h"

namespace tpm {
namespace pmk {

// Mesh geometry: point i of an axis sits at lo + i h; `box` > 0 wraps
// positions periodically into [0, box) (lo = 0 then), `box` = 0 leaves them
// (the isolated mesh, where every position lies well inside the mesh).
struct MeshGeom {
    double lo[3];
    double box;
    double h;
    int ng;  // points per axis of the transformed mesh
};

// Mesh force F = -grad Phi and potential P at the particle of curve-order slot
// s: CIC weights of its position, and at each of the eight mesh points the
// four-point difference of the potential along each axis (coefficients 2/3
// and 1/12; the sum over the corners divided by h once), everything in
// double.
// LEAN: the eight corners one after the other, not unrolled (the same
// operations in the same order, fewer live registers), for kernels whose
// other work sets their register budget.
template <typename T, bool LEAN = false>
__device__ __forceinline__ void interp_at(const double *__restrict__ ps, int64_t n, int64_t s,
                                          const T *__restrict__ phi, const MeshGeom &mg,
                                          double F[3], double &P) {
    const double box = mg.box, h = mg.h;
    const int ng = mg.ng;
    int i0[3];
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double u = ps[(size_t)a * n + s] - mg.lo[a];
        if (box > 0.0) {
            if (u < 0.0)
                u += box;
            if (u >= box)
                u -= box;
        }
        const double f = u / h;
        const double fl = floor(f);
        w[a] = f - fl;
        // any input (even outside the box or NaN) stays on the mesh
        int i = (int)fmin(fmax(fl, -1.0e9), 1.0e9) % ng;
        if (i < 0)
            i += ng;
        i0[a] = i;
    }
    const int mask = ng - 1;
    auto at = [&](int x, int y, int z) -> double {
        return (double)phi[((size_t)(x & mask) * ng + (y & mask)) * ng + (z & mask)];
    };
    F[0] = F[1] = F[2] = 0.0;
    P = 0.0;
    auto corner = [&](int c) {
        double wt = 1.0;
        int t[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int up = (c >> (2 - a)) & 1;
            wt *= up ? w[a] : 1.0 - w[a];
            t[a] = i0[a] + up;
        }
        // -grad Phi at mesh point t, times h (the division by h follows the sum)
        {
            const double g = ((2.0 / 3.0) * (at(t[0] + 1, t[1], t[2]) - at(t[0] - 1, t[1], t[2])) -
                              (1.0 / 12.0) * (at(t[0] + 2, t[1], t[2]) - at(t[0] - 2, t[1], t[2])));
            F[0] += wt * -g;
        }
        {
            const double g = ((2.0 / 3.0) * (at(t[0], t[1] + 1, t[2]) - at(t[0], t[1] - 1, t[2])) -
                              (1.0 / 12.0) * (at(t[0], t[1] + 2, t[2]) - at(t[0], t[1] - 2, t[2])));
            F[1] += wt * -g;
        }
        {
            const double g = ((2.0 / 3.0) * (at(t[0], t[1], t[2] + 1) - at(t[0], t[1], t[2] - 1)) -
                              (1.0 / 12.0) * (at(t[0], t[1], t[2] + 2) - at(t[0], t[1], t[2] - 2)));
            F[2] += wt * -g;
        }
        P += wt * at(t[0], t[1], t[2]);
    };
    if constexpr (LEAN) {
#pragma unroll 1
        for (int c = 0; c < 8; c++)
            corner(c);
    } else {
#pragma unroll
        for (int c = 0; c < 8; c++)
            corner(c);
    }
    F[0] /= h;
    F[1] /= h;
    F[2] /= h;
}

// Mesh geometry of the current build (host, pm.hip).
MeshGeom mesh_geom(const tpm_ctx *c);

}  // namespace pmk
}  // namespace tpm
