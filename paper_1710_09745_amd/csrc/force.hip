// Link force: the gradient of the solve's loss with respect to the fat and long
// links (the backward of X = A^{-1} B; derived from dA = -(dD_eo D_oe + D_eo dD_oe)
// and D_eo^H = -D_oe).  For a link W_mu(x) of hop length k, y = x + k mu:
//   x even: grad = +eta_mu(x) sum_i [ Lam_i(x) Y_X,i(y)^H + X_i(x) Y_L,i(y)^H ]
//   x odd : grad = -eta_mu(x) sum_i [ Y_X,i(x) Lam_i(y)^H + Y_L,i(x) X_i(y)^H ]
// with Y_X = D_oe X, Y_L = D_oe Lam on the odd sites.  One thread per
// (site, direction) accumulates the outer products of all N columns for the
// fat (and long) link of that site; output in the canonical [4][V][3][3] layout.
#include "device_common.h"
#include "internal.h"

namespace bcg {

__global__ void __launch_bounds__(256)
k_link_force(const double2* __restrict__ X, const double2* __restrict__ Lam,
             const double2* __restrict__ YX, const double2* __restrict__ YL, int N, Geom g,
             int improved, double2* __restrict__ gfat, double2* __restrict__ glong) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    const int p = blockIdx.z;
    if (i >= g.Vh) return;
    int x[4];
    site_coords(g, i, p, x);
    const long Vh = g.Vh;
    const long V = 2 * Vh;
    const long lex = x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * (x[2] + (long)g.L[2] * x[3]));
    // fields at x (parity p) and at y (parity 1-p)
    const double2* U1 = p == 0 ? Lam : YX;
    const double2* U2 = p == 0 ? X : YL;
    const double2* V1 = p == 0 ? YX : Lam;
    const double2* V2 = p == 0 ? YL : X;
    const double s = (double)eta_sign(x, mu) * (p == 0 ? 1.0 : -1.0);
    for (int k = 1; k <= (improved ? 3 : 1); k += 2) {
        const int y = neighbour_cb(g, x, mu, k);
        C2<double> acc[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) acc[e] = C2<double>{0.0, 0.0};
        for (int r = 0; r < N; ++r) {
            C2<double> u1[3], u2[3], v1[3], v2[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long ox = ((long)r * 3 + c) * Vh + i, oy = ((long)r * 3 + c) * Vh + y;
                u1[c] = ld(U1 + ox);
                u2[c] = ld(U2 + ox);
                v1[c] = ld(V1 + oy);
                v2[c] = ld(V2 + oy);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    // u v^H: (a, b) = u_a conj(v_b) = conj(v_b) u_a
                    cmac_conj(acc[3 * a + b], v1[b], u1[a]);
                    cmac_conj(acc[3 * a + b], v2[b], u2[a]);
                }
        }
        double2* out = (k == 1 ? gfat : glong) + ((long)mu * V + lex) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) out[e] = make_double2(s * acc[e].re, s * acc[e].im);
    }
}

hipError_t launch_link_force(const double2* X, const double2* Lam, const double2* YX,
                             const double2* YL, int N, const Geom& g, int improved,
                             double2* gfat, double2* glong, hipStream_t s) {
    dim3 grid((g.Vh + 255) / 256, 4, 2);
    hipLaunchKernelGGL(k_link_force, grid, dim3(256), 0, s, X, Lam, YX, YL, N, g, improved, gfat, glong);
    return hipGetLastError();
}

}  // namespace bcg
