/*
 * CPU FP64 oracle for the staggered stencil, the even-odd normal operator and
 * the link force.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
 * bench's CPU-baseline leg call it; the solver library never does.
 *
 * Plain C99 complex arithmetic, one OpenMP loop over output sites, no
 * blocking or reordering beyond what the definitions say.
 *
 * Conventions (fixed here because the paper leaves them open):
 *   dims = (Lx, Ly, Lz, Lt), every extent even, periodic boundaries.
 *   lex(x) = x0 + Lx*(x1 + Ly*(x2 + Lz*x3)), parity = (x0+x1+x2+x3) mod 2,
 *   checkerboard index cb = lex >> 1.
 *   links [4][V][3][3]: U_mu(x) at [mu][lex(x)], acting as (U v)_a = sum_b U_ab v_b.
 *   eta_0 = 1, eta_1 = (-1)^x0, eta_2 = (-1)^(x0+x1), eta_3 = (-1)^(x0+x1+x2).
 *
 * Staggered operator (Sec. 3.2, Eq. 2, read with the standard staggered phases
 * and an anti-Hermitian hopping term, no 1/2 prefactor):
 *   (D psi)(x) = sum_mu eta_mu(x) [ F_mu(x) psi(x+mu) - F_mu(x-mu)^H psi(x-mu)
 *                                 + G_mu(x) psi(x+3mu) - G_mu(x-3mu)^H psi(x-3mu) ]
 * with fat links F (one hop) and long links G (three hops); the naive operator
 * drops the G terms.  Mass enters as 2m: (2m + D)^H (2m + D) = 4m^2 - D^2, whose
 * even-even block is A = 4 m^2 - D_eo D_oe, the Schur-reduced normal operator
 * (Sec. 3.2) that the block solver inverts.
 */
#include <complex.h>
#include <stddef.h>
#include <string.h>

typedef double complex cplx;

/* threads only pay off on lattices of a few thousand sites or more */
#define PAR_OK (vol(dims) >= 8192)

static long vol(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords_of(const int d[4], long lex, int c[4]) {
    c[0] = (int)(lex % d[0]); lex /= d[0];
    c[1] = (int)(lex % d[1]); lex /= d[1];
    c[2] = (int)(lex % d[2]); lex /= d[2];
    c[3] = (int)lex;
}

static long lex_of(const int d[4], const int c[4]) {
    return c[0] + (long)d[0] * (c[1] + (long)d[1] * (c[2] + (long)d[2] * c[3]));
}

static int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* staggered phase eta_mu(x) */
static double eta(int mu, const int c[4]) {
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* lex index of x + k*mu (k may be negative), periodic */
static long shift(const int d[4], const int c[4], int mu, int k) {
    int y[4] = {c[0], c[1], c[2], c[3]};
    y[mu] = ((y[mu] + k) % d[mu] + d[mu]) % d[mu];
    return lex_of(d, y);
}

/* lex index of the site with checkerboard index cb and the given parity */
static long lex_from_cb(const int d[4], long cb, int parity) {
    long l = 2 * cb;
    int c[4];
    coords_of(d, l, c);
    if (parity_of(c) != parity) l += 1;
    return l;
}

/* out += s * U v   and   out += s * U^H v  (U row-major 3x3) */
static void mv_acc(cplx *out, double s, const cplx *U, const cplx *v) {
    for (int a = 0; a < 3; ++a) {
        cplx t = 0;
        for (int b = 0; b < 3; ++b) t += U[3 * a + b] * v[b];
        out[a] += s * t;
    }
}
static void mhv_acc(cplx *out, double s, const cplx *U, const cplx *v) {
    for (int a = 0; a < 3; ++a) {
        cplx t = 0;
        for (int b = 0; b < 3; ++b) t += conj(U[3 * b + a]) * v[b];
        out[a] += s * t;
    }
}

/* (D psi)(x) at one site of the full lattice; psi indexed by lex */
static void dslash_site(const int d[4], int improved, const cplx *fat, const cplx *lng,
                        const cplx *psi, long x, cplx out[3]) {
    const long V = vol(d);
    int c[4];
    coords_of(d, x, c);
    out[0] = out[1] = out[2] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const double e = eta(mu, c);
        const long xf = shift(d, c, mu, +1), xb = shift(d, c, mu, -1);
        mv_acc(out, e, fat + 9 * ((long)mu * V + x), psi + 3 * xf);
        mhv_acc(out, -e, fat + 9 * ((long)mu * V + xb), psi + 3 * xb);
        if (improved) {
            const long yf = shift(d, c, mu, +3), yb = shift(d, c, mu, -3);
            mv_acc(out, e, lng + 9 * ((long)mu * V + x), psi + 3 * yf);
            mhv_acc(out, -e, lng + 9 * ((long)mu * V + yb), psi + 3 * yb);
        }
    }
}

/* Full-lattice D: psi, out are [V][3] in lex order. */
void oracle_dslash_full(const int dims[4], int improved, const cplx *fat, const cplx *lng,
                        const cplx *psi, cplx *out) {
    const long V = vol(dims);
#pragma omp parallel for schedule(static) if (PAR_OK)
    for (long x = 0; x < V; ++x) dslash_site(dims, improved, fat, lng, psi, x, out + 3 * x);
}

/* (D psi)(x) for x of parity p, psi a field on the opposite checkerboard ([V/2][3], cb order) */
static void hop_site(const int d[4], int improved, const cplx *fat, const cplx *lng,
                     const cplx *psi, long x, cplx out[3]) {
    const long V = vol(d);
    int c[4];
    coords_of(d, x, c);
    out[0] = out[1] = out[2] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const double e = eta(mu, c);
        const long xf = shift(d, c, mu, +1), xb = shift(d, c, mu, -1);
        mv_acc(out, e, fat + 9 * ((long)mu * V + x), psi + 3 * (xf >> 1));
        mhv_acc(out, -e, fat + 9 * ((long)mu * V + xb), psi + 3 * (xb >> 1));
        if (improved) {
            const long yf = shift(d, c, mu, +3), yb = shift(d, c, mu, -3);
            mv_acc(out, e, lng + 9 * ((long)mu * V + x), psi + 3 * (yf >> 1));
            mhv_acc(out, -e, lng + 9 * ((long)mu * V + yb), psi + 3 * (yb >> 1));
        }
    }
}

/*
 * One checkerboard hop: out = D_{p, 1-p} in, for nrhs fields.
 * in: [nrhs][V/2][3] on parity 1-p, out: [nrhs][V/2][3] on parity p.
 */
void oracle_hop(const int dims[4], int improved, const cplx *fat, const cplx *lng,
                int out_parity, int nrhs, const cplx *in, cplx *out) {
    const long Vh = vol(dims) / 2;
    for (int r = 0; r < nrhs; ++r) {
        const cplx *src = in + (long)r * Vh * 3;
        cplx *dst = out + (long)r * Vh * 3;
#pragma omp parallel for schedule(static) if (PAR_OK)
        for (long i = 0; i < Vh; ++i) {
            const long x = lex_from_cb(dims, i, out_parity);
            hop_site(dims, improved, fat, lng, src, x, dst + 3 * i);
        }
    }
}

/*
 * A = 4 m^2 - D_eo D_oe on even fields: out = A in, [nrhs][V/2][3].
 * work: caller-provided [nrhs][V/2][3] scratch for the odd intermediate.
 */
void oracle_apply(const int dims[4], int improved, const cplx *fat, const cplx *lng,
                  double mass, int nrhs, const cplx *in, cplx *out, cplx *work) {
    const long n = (long)nrhs * (vol(dims) / 2) * 3;
    oracle_hop(dims, improved, fat, lng, 1, nrhs, in, work);
    oracle_hop(dims, improved, fat, lng, 0, nrhs, work, out);
    const double m2 = 4.0 * mass * mass;
    for (long k = 0; k < n; ++k) out[k] = m2 * in[k] - out[k];
}

/*
 * (A in)(x) at selected even sites only, one site at a time:
 *   (A in)(x) = 4 m^2 in(x) - sum over the 16 hops of x of  +/-eta W (D_oe in)(y).
 * cb: nsites even-site checkerboard indices; out: [nrhs][nsites][3].
 */
void oracle_apply_sites(const int dims[4], int improved, const cplx *fat, const cplx *lng,
                        double mass, int nrhs, const cplx *in, long nsites, const long *cb,
                        cplx *out) {
    const long V = vol(dims), Vh = V / 2;
    const double m2 = 4.0 * mass * mass;
#pragma omp parallel for schedule(dynamic) if (nsites * nrhs >= 64)
    for (long s = 0; s < nsites; ++s) {
        const long x = lex_from_cb(dims, cb[s], 0);
        int c[4];
        coords_of(dims, x, c);
        for (int r = 0; r < nrhs; ++r) {
            const cplx *src = in + (long)r * Vh * 3;
            cplx acc[3] = {0, 0, 0};
            for (int mu = 0; mu < 4; ++mu) {
                const double e = eta(mu, c);
                for (int k = 1; k <= (improved ? 3 : 1); k += 2) {
                    const cplx *lk = (k == 1) ? fat : lng;
                    const long yf = shift(dims, c, mu, +k), yb = shift(dims, c, mu, -k);
                    cplx t[3];
                    hop_site(dims, improved, fat, lng, src, yf, t);
                    mv_acc(acc, e, lk + 9 * ((long)mu * V + x), t);
                    hop_site(dims, improved, fat, lng, src, yb, t);
                    mhv_acc(acc, -e, lk + 9 * ((long)mu * V + yb), t);
                }
            }
            cplx *dst = out + ((long)r * nsites + s) * 3;
            for (int a = 0; a < 3; ++a) dst[a] = m2 * src[3 * cb[s] + a] - acc[a];
        }
    }
}

/*
 * Link force for L with dL = -Re sum_i Lam_i^H dA X_i  (A = 4m^2 - D_eo D_oe).
 * X, Lam: even fields [nrhs][V/2][3]; YX = D_oe X, YL = D_oe Lam: odd fields.
 * For a link W_mu(x) of hop length k (1 fat, 3 long), y = x + k mu:
 *   x even:  grad W_mu(x) = +eta_mu(x) sum_i [ Lam_i(x) YX_i(y)^H + X_i(x) YL_i(y)^H ]
 *   x odd :  grad W_mu(x) = -eta_mu(x) sum_i [ YX_i(x) Lam_i(y)^H + YL_i(x) X_i(y)^H ]
 * (derived from dA = -(dD_eo D_oe + D_eo dD_oe) and D_eo^H = -D_oe; gradient in
 * the complex convention dL/dRe + i dL/dIm).  Outputs [4][V][3][3], overwritten;
 * glong is ignored when improved == 0.
 */
void oracle_link_force(const int dims[4], int improved, int nrhs, const cplx *X, const cplx *Lam,
                       const cplx *YX, const cplx *YL, cplx *gfat, cplx *glong) {
    const long V = vol(dims), Vh = V / 2;
#pragma omp parallel for schedule(static) if (PAR_OK)
    for (long x = 0; x < V; ++x) {
        int c[4];
        coords_of(dims, x, c);
        const int p = parity_of(c);
        for (int mu = 0; mu < 4; ++mu) {
            const double e = eta(mu, c);
            for (int k = 1; k <= (improved ? 3 : 1); k += 2) {
                cplx *g = ((k == 1) ? gfat : glong) + 9 * ((long)mu * V + x);
                const long y = shift(dims, c, mu, +k);
                const long ix = x >> 1, iy = y >> 1;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        cplx s = 0;
                        for (int r = 0; r < nrhs; ++r) {
                            const long o = (long)r * Vh * 3;
                            if (p == 0)
                                s += Lam[o + 3 * ix + a] * conj(YX[o + 3 * iy + b]) +
                                     X[o + 3 * ix + a] * conj(YL[o + 3 * iy + b]);
                            else
                                s += YX[o + 3 * ix + a] * conj(Lam[o + 3 * iy + b]) +
                                     YL[o + 3 * ix + a] * conj(X[o + 3 * iy + b]);
                        }
                        g[3 * a + b] = (p == 0 ? e : -e) * s;
                    }
            }
        }
    }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
