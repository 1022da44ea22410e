/*
 * gke_oracle.c -- plain FP64 CPU oracle for the GKE two-point statistics.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP path (no headers, tables, helpers or generators).
 *
 * It follows the paper's method in the paper's order (Gatti et al., "An
 * efficient numerical method for the Generalised Kolmogorov Equation"):
 *
 *   Step 1 (Section "Step 1"): means U,V,W,P over all grid points and
 *     snapshots; mean shear dU/dy with the five-point stencil; one-point
 *     moments of the fluctuations, pseudo-dissipation eps = nu<du_i/dx_j du_i/dx_j>
 *     (definition below eq. GKE).
 *   Step 2 (Sections "Products instead of correlations" and "Step 2"): each
 *     GKE term is written as a sum of two-point correlations (eq. expansion
 *     and its analogues); every correlation <A(x,Y1,z) B(x+rx,Y2,z+rz)>
 *     is computed through the Parseval identity as the inverse transform of
 *     conj(A^(Y1)) B^(Y2), averaged over snapshots; triple correlations use
 *     in-plane products formed in physical space.
 *   Step 3 (Section "Step 3"): wall-normal derivatives are taken by the
 *     Python wrapper with the five-point weights exported here.
 *
 * Conventions (readings where the paper is silent, listed in the design notes):
 *   forward transform A^(k) = (1/(Nx Nz)) sum A e^{-i(alpha x + beta z)};
 *   correlation C[A,B](r) = sum_k conj(A^(k;Y1)) B^(k;Y2) e^{+i(alpha rx + beta rz)};
 *   the full (Nx x Nz) complex spectrum is kept -- no half-spectrum weights;
 *   spectral derivatives use i*alpha, i*beta with the Nyquist multiplier 0.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Own plain FFT: recursive decimation in time over the smallest prime       */
/* factor.  out[k] = sum_n in[n*stride] exp(sign*2*pi*i*n*k/n_len).         */
/* ------------------------------------------------------------------------ */
static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

static cplx unit_root(long num, long den, int sign)
{
    /* exp(sign * 2 pi i num/den), num reduced mod den */
    long r = num % den;
    if (r < 0) r += den;
    double a = 2.0 * M_PI * (double)r / (double)den;
    return cos(a) + (double)sign * sin(a) * I;
}

/* root[t * rs] = exp(sign 2 pi i t/n) for t < n; work must hold n elements */
static void dft_rec(int n, const cplx *in, long stride, cplx *out, const cplx *root, long rs,
                    cplx *work)
{
    if (n == 1) { out[0] = in[0]; return; }
    int p = smallest_factor(n);
    int m = n / p;
    /* sub-transforms of the p decimated sequences (their roots: every p-th) */
    for (int q = 0; q < p; ++q)
        dft_rec(m, in + q * stride, stride * p, out + q * m, root, rs * p, work);
    /* combine: X[k] = sum_q w^{q k} Y_q[k mod m], w = exp(sign 2 pi i/n) */
    for (int k = 0; k < n; ++k) {
        cplx acc = 0.0;
        for (int q = 0; q < p; ++q)
            acc += root[(((long)q * k) % n) * rs] * out[q * m + (k % m)];
        work[k] = acc;
    }
    memcpy(out, work, sizeof(cplx) * (size_t)n);
}

/* 1-D transform of a strided complex sequence, result written back in place */
static void fft1(int n, cplx *data, long stride, int sign, cplx *buf /* 4n */)
{
    cplx *in = buf, *out = buf + n, *work = buf + 2 * n, *root = buf + 3 * n;
    for (int t = 0; t < n; ++t) root[t] = unit_root(t, n, sign);
    for (int i = 0; i < n; ++i) in[i] = data[i * stride];
    dft_rec(n, in, 1, out, root, 1, work);
    for (int i = 0; i < n; ++i) data[i * stride] = out[i];
}

/* 2-D transform of a [nz][nx] complex plane; x rows then z columns */
static void fft2(int nx, int nz, cplx *plane, int sign, cplx *buf)
{
    for (int z = 0; z < nz; ++z) fft1(nx, plane + (long)z * nx, 1, sign, buf);
    for (int x = 0; x < nx; ++x) fft1(nz, plane + x, nx, sign, buf);
}

/* thread count of the OpenMP regions (the CPU-baseline timing states it) */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* exported for the tests: plain 1-D transform of n complex values */
int or_fft1(int n, const double *in_ri, double *out_ri, int sign)
{
    if (n < 1) return 1;
    cplx *d = malloc(sizeof(cplx) * (size_t)n);
    cplx *buf = malloc(sizeof(cplx) * 4 * (size_t)n);
    for (int i = 0; i < n; ++i) d[i] = in_ri[2 * i] + in_ri[2 * i + 1] * I;
    fft1(n, d, 1, sign, buf);
    for (int i = 0; i < n; ++i) { out_ri[2 * i] = creal(d[i]); out_ri[2 * i + 1] = cimag(d[i]); }
    free(d); free(buf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Five-point first-derivative weights on the nonuniform y grid (Section    */
/* "Step 3": explicit, non-compact, five-point stencil).  Written as the    */
/* derivative of the Lagrange interpolant through five nodes: centred in    */
/* the interior, shifted to the five nodes nearest each wall.  D is the     */
/* dense [ny][ny] matrix.                                                   */
/* ------------------------------------------------------------------------ */
int or_fd5(int ny, const double *y, double *D)
{
    if (ny < 5) return 1;
    memset(D, 0, sizeof(double) * (size_t)ny * ny);
    for (int j = 0; j < ny; ++j) {
        int j0 = j - 2;
        if (j0 < 0) j0 = 0;
        if (j0 > ny - 5) j0 = ny - 5;
        for (int a = 0; a < 5; ++a) {
            int m = j0 + a;
            /* L_m'(y_j) = sum_{l != m} 1/(y_m - y_l) prod_{n != m,l} (y_j - y_n)/(y_m - y_n) */
            double s = 0.0;
            for (int b = 0; b < 5; ++b) {
                int l = j0 + b;
                if (l == m) continue;
                double t = 1.0 / (y[m] - y[l]);
                for (int c = 0; c < 5; ++c) {
                    int n = j0 + c;
                    if (n == m || n == l) continue;
                    t *= (y[j] - y[n]) / (y[m] - y[n]);
                }
                s += t;
            }
            D[(long)j * ny + m] = s;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 1: means and one-point statistics.                                  */
/* snap layout: [ns][4][ny][nz][nx], fields (u~, v~, w~, p~).                */
/* ------------------------------------------------------------------------ */
#define FLD(snap, s, f, j) ((snap) + ((((long)(s) * 4 + (f)) * ny + (j)) * (long)nz * nx))

int or_means(int nx, int ny, int nz, int ns, const double *snap, double *means /* [4][ny] */)
{
    long npl = (long)nx * nz;
    for (int f = 0; f < 4; ++f)
        for (int j = 0; j < ny; ++j) {
            double acc = 0.0;
            for (int s = 0; s < ns; ++s) {
                const double *pl = FLD(snap, s, f, j);
                for (long i = 0; i < npl; ++i) acc += pl[i];
            }
            means[f * ny + j] = acc / ((double)ns * (double)npl);
        }
    return 0;
}

/* profile rows */
enum { P_U, P_V, P_W, P_P, P_S, P_Q, P_UV, P_PV, P_TX, P_TY, P_TZ, P_EPS, NPROF };

static double kx_mult(int k, int n, double len)
{
    /* alpha for index k of an n-point periodic grid; Nyquist -> 0 */
    if (2 * k == n) return 0.0;
    int kk = (k <= n / 2) ? k : k - n;
    return 2.0 * M_PI * (double)kk / len;
}

int or_onepoint(int nx, int ny, int nz, int ns, const double *snap, const double *means,
                const double *D, double lx, double lz, double nu, const int *mask,
                double *prof /* [NPROF][ny] */)
{
    long npl = (long)nx * nz;
    memset(prof, 0, sizeof(double) * NPROF * (size_t)ny);
    for (int f = 0; f < 4; ++f)
        for (int j = 0; j < ny; ++j) prof[f * ny + j] = means[f * ny + j];
    for (int j = 0; j < ny; ++j) {
        double s = 0.0;
        for (int m = 0; m < ny; ++m) s += D[(long)j * ny + m] * means[m];
        prof[P_S * ny + j] = s;
    }
    int nmax = nx > nz ? nx : nz;
    double norm = 1.0 / ((double)ns * (double)npl);
    /* planes are independent; mask (optional) selects the planes to compute */
    #pragma omp parallel
    {
    cplx *buf = malloc(sizeof(cplx) * 4 * (size_t)nmax);
    cplx *pl = malloc(sizeof(cplx) * (size_t)npl);
    cplx *dp = malloc(sizeof(cplx) * (size_t)npl);
    double *dfl = malloc(sizeof(double) * (size_t)npl);
    #pragma omp for schedule(dynamic)
    for (int j = 0; j < ny; ++j) {
        if (mask && !mask[j]) continue;
        double aq = 0, auv = 0, apv = 0, atx = 0, aty = 0, atz = 0, aeps = 0;
        for (int s = 0; s < ns; ++s) {
            const double *uu = FLD(snap, s, 0, j), *vv = FLD(snap, s, 1, j);
            const double *ww = FLD(snap, s, 2, j), *pp = FLD(snap, s, 3, j);
            for (long i = 0; i < npl; ++i) {
                double u = uu[i] - means[0 * ny + j], v = vv[i] - means[1 * ny + j];
                double w = ww[i] - means[2 * ny + j], p = pp[i] - means[3 * ny + j];
                double q = u * u + v * v + w * w;
                aq += q; auv += u * v; apv += p * v;
                atx += q * u; aty += q * v; atz += q * w;
            }
            /* pseudo-dissipation: x and z derivatives spectral, y derivative FD5 */
            for (int c = 0; c < 3; ++c) {
                const double *src = FLD(snap, s, c, j);
                double mu = means[c * ny + j];
                for (long i = 0; i < npl; ++i) pl[i] = src[i] - mu;
                fft2(nx, nz, pl, -1, buf);
                for (long i = 0; i < npl; ++i) pl[i] /= (double)npl;
                for (int dir = 0; dir < 2; ++dir) {
                    for (int z = 0; z < nz; ++z)
                        for (int x = 0; x < nx; ++x) {
                            double k = dir == 0 ? kx_mult(x, nx, lx) : kx_mult(z, nz, lz);
                            dp[(long)z * nx + x] = I * k * pl[(long)z * nx + x];
                        }
                    fft2(nx, nz, dp, +1, buf);
                    for (long i = 0; i < npl; ++i) aeps += creal(dp[i]) * creal(dp[i]);
                }
                /* d/dy with the five-point weights */
                for (long i = 0; i < npl; ++i) dfl[i] = 0.0;
                for (int m = 0; m < ny; ++m) {
                    double wgt = D[(long)j * ny + m];
                    if (wgt == 0.0) continue;
                    const double *sm = FLD(snap, s, c, m);
                    double mm = means[c * ny + m];
                    for (long i = 0; i < npl; ++i) dfl[i] += wgt * (sm[i] - mm);
                }
                for (long i = 0; i < npl; ++i) aeps += dfl[i] * dfl[i];
            }
        }
        prof[P_Q * ny + j] = aq * norm;
        prof[P_UV * ny + j] = auv * norm;
        prof[P_PV * ny + j] = apv * norm;
        prof[P_TX * ny + j] = atx * norm;
        prof[P_TY * ny + j] = aty * norm;
        prof[P_TZ * ny + j] = atz * norm;
        prof[P_EPS * ny + j] = nu * aeps * norm;
    }
    free(buf); free(pl); free(dp); free(dfl);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 2: two-point correlations for a list of ordered (Y1, Y2) pairs.      */
/* ------------------------------------------------------------------------ */
/* fields transformed per plane: fluctuations and in-plane products */
enum { F_U, F_V, F_W, F_P, F_UU, F_VV, F_WW, F_UV, F_UW, F_VW, F_Q, NF };

/* product field index of u_i u_j */
static int prod_index(int i, int j)
{
    static const int tab[3][3] = { { F_UU, F_UV, F_UW }, { F_UV, F_VV, F_VW }, { F_UW, F_VW, F_WW } };
    return tab[i][j];
}

/* correlation list: C[A,B] with A at Y1, B at Y2 */
enum {
    C_UU, C_VV, C_WW,             /* C[u_i,u_i] */
    C_QU, C_QV, C_QW,             /* C[q,u_j] */
    C_UQ, C_VQ, C_WQ,             /* C[u_j,q] */
    C_PV, C_VP, C_UV, C_VU,       /* C[p,v] C[v,p] C[u,v] C[v,u] */
    C_PIJ_UI,                     /* 9: C[u_i u_j, u_i] at C_PIJ_UI + 3*j + i */
    C_UI_PIJ = C_PIJ_UI + 9,      /* 9: C[u_i, u_i u_j] at C_UI_PIJ + 3*j + i */
    NCORR = C_UI_PIJ + 9
};

static void corr_fields(int c, int *a, int *b)
{
    switch (c) {
    case C_UU: *a = F_U; *b = F_U; return;
    case C_VV: *a = F_V; *b = F_V; return;
    case C_WW: *a = F_W; *b = F_W; return;
    case C_QU: *a = F_Q; *b = F_U; return;
    case C_QV: *a = F_Q; *b = F_V; return;
    case C_QW: *a = F_Q; *b = F_W; return;
    case C_UQ: *a = F_U; *b = F_Q; return;
    case C_VQ: *a = F_V; *b = F_Q; return;
    case C_WQ: *a = F_W; *b = F_Q; return;
    case C_PV: *a = F_P; *b = F_V; return;
    case C_VP: *a = F_V; *b = F_P; return;
    case C_UV: *a = F_U; *b = F_V; return;
    case C_VU: *a = F_V; *b = F_U; return;
    default: break;
    }
    if (c >= C_PIJ_UI && c < C_PIJ_UI + 9) {
        int j = (c - C_PIJ_UI) / 3, i = (c - C_PIJ_UI) % 3;
        *a = prod_index(i, j); *b = F_U + i;
    } else {
        int j = (c - C_UI_PIJ) / 3, i = (c - C_UI_PIJ) % 3;
        *a = F_U + i; *b = prod_index(i, j);
    }
}

/* output term slots T1..T14 -> 0..13 */
enum { T1, T2, T3, T4, T5, T6, T7, T8, T9, T10, T11, T12, T13, T14, NT };

int or_pairs(int nx, int ny, int nz, int ns, const double *snap, const double *prof,
             double lx, double lz, double nu, int npairs, const int *py1, const int *py2,
             double *out /* [npairs][NT][nz][nx] */, int nthreads)
{
    long npl = (long)nx * nz;
    int nmax = nx > nz ? nx : nz;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* planes touched by the pair list */
    int *slot = malloc(sizeof(int) * (size_t)ny);
    for (int j = 0; j < ny; ++j) slot[j] = -1;
    int nplanes = 0;
    for (int k = 0; k < npairs; ++k) {
        if (py1[k] < 0 || py1[k] >= ny || py2[k] < 0 || py2[k] >= ny) { free(slot); return 1; }
        if (slot[py1[k]] < 0) slot[py1[k]] = nplanes++;
        if (slot[py2[k]] < 0) slot[py2[k]] = nplanes++;
    }
    int *plane_of = malloc(sizeof(int) * (size_t)(nplanes > 0 ? nplanes : 1));
    for (int j = 0; j < ny; ++j) if (slot[j] >= 0) plane_of[slot[j]] = j;

    /* per-snapshot spectra of the NF fields on each touched plane */
    cplx *spec = malloc(sizeof(cplx) * (size_t)nplanes * NF * npl);
    /* per-pair correlation spectra accumulated over snapshots */
    cplx *acc = calloc((size_t)npairs * NCORR * npl, sizeof(cplx));
    if (!spec || !acc) { free(slot); free(plane_of); free(spec); free(acc); return 2; }

    for (int s = 0; s < ns; ++s) {
        /* fluctuations, in-plane products in physical space, forward transforms */
        #pragma omp parallel
        {
            cplx *buf = malloc(sizeof(cplx) * 4 * (size_t)nmax);
            #pragma omp for schedule(dynamic)
            for (int t = 0; t < nplanes * NF; ++t) {
                int pi = t / NF, f = t % NF, j = plane_of[pi];
                cplx *dst = spec + ((long)pi * NF + f) * npl;
                const double *u = FLD(snap, s, 0, j), *v = FLD(snap, s, 1, j);
                const double *w = FLD(snap, s, 2, j), *p = FLD(snap, s, 3, j);
                double U = prof[P_U * ny + j], V = prof[P_V * ny + j];
                double W = prof[P_W * ny + j], P = prof[P_P * ny + j];
                for (long i = 0; i < npl; ++i) {
                    double a = u[i] - U, b = v[i] - V, c = w[i] - W, d = p[i] - P, val;
                    switch (f) {
                    case F_U: val = a; break;
                    case F_V: val = b; break;
                    case F_W: val = c; break;
                    case F_P: val = d; break;
                    case F_UU: val = a * a; break;
                    case F_VV: val = b * b; break;
                    case F_WW: val = c * c; break;
                    case F_UV: val = a * b; break;
                    case F_UW: val = a * c; break;
                    case F_VW: val = b * c; break;
                    default: val = a * a + b * b + c * c; break;
                    }
                    dst[i] = val;
                }
                fft2(nx, nz, dst, -1, buf);
                for (long i = 0; i < npl; ++i) dst[i] /= (double)npl;
            }
            free(buf);
        }
        /* Parseval: accumulate conj(A^(Y1)) B^(Y2) for every needed correlation */
        #pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < npairs * NCORR; ++t) {
            int k = t / NCORR, c = t % NCORR, fa, fb;
            corr_fields(c, &fa, &fb);
            const cplx *A = spec + ((long)slot[py1[k]] * NF + fa) * npl;
            const cplx *B = spec + ((long)slot[py2[k]] * NF + fb) * npl;
            cplx *dst = acc + ((long)k * NCORR + c) * npl;
            for (long i = 0; i < npl; ++i) dst[i] += conj(A[i]) * B[i];
        }
    }
    free(spec);

    /* average, inverse transform, assembly */
    #pragma omp parallel
    {
        cplx *buf = malloc(sizeof(cplx) * 4 * (size_t)nmax);
        double *C = malloc(sizeof(double) * NCORR * (size_t)npl);
        cplx *tmp = malloc(sizeof(cplx) * (size_t)npl);
        #pragma omp for schedule(dynamic)
        for (int k = 0; k < npairs; ++k) {
            int j1 = py1[k], j2 = py2[k];
            for (int c = 0; c < NCORR; ++c) {
                cplx *a = acc + ((long)k * NCORR + c) * npl;
                for (long i = 0; i < npl; ++i) tmp[i] = a[i] / (double)ns;
                fft2(nx, nz, tmp, +1, buf);
                for (long i = 0; i < npl; ++i) C[(long)c * npl + i] = creal(tmp[i]);
            }
#define PR(row, j) prof[(row) * ny + (j)]
            double q1 = PR(P_Q, j1), q2 = PR(P_Q, j2);
            double dU = PR(P_U, j2) - PR(P_U, j1);
            double Tj1[3] = { PR(P_TX, j1), PR(P_TY, j1), PR(P_TZ, j1) };
            double Tj2[3] = { PR(P_TX, j2), PR(P_TY, j2), PR(P_TZ, j2) };
            double Sstar = 0.5 * (PR(P_S, j1) + PR(P_S, j2));
            double dS = PR(P_S, j2) - PR(P_S, j1);
            double *o = out + (long)k * NT * npl;
            memset(o, 0, sizeof(double) * NT * (size_t)npl);
            for (long i = 0; i < npl; ++i) {
#define CC(c) C[(long)(c) * npl + i]
                double R = CC(C_UU) + CC(C_VV) + CC(C_WW);
                /* scale energy <du^2> (eq. du2) via the correlation expansion */
                double t1 = q1 + q2 - 2.0 * R;
                o[T1 * npl + i] = t1;
                /* mean-flow part of the scale flux: <du^2 dU> */
                o[T3 * npl + i] = dU * t1;
                /* turbulent scale fluxes <du^2 du_j>, j = x, y, z */
                for (int j = 0; j < 3; ++j) {
                    double sum = Tj2[j] - Tj1[j] + CC(C_QU + j) - CC(C_UQ + j);
                    for (int ii = 0; ii < 3; ++ii)
                        sum += 2.0 * (CC(C_PIJ_UI + 3 * j + ii) - CC(C_UI_PIJ + 3 * j + ii));
                    o[(j == 0 ? T2 : j == 1 ? T5 : T7) * npl + i] = sum;
                }
                /* turbulent spatial flux <v* du^2> */
                {
                    double sum = Tj1[1] + Tj2[1] + CC(C_VQ) + CC(C_QV);
                    for (int ii = 0; ii < 3; ++ii)
                        sum -= 2.0 * (CC(C_PIJ_UI + 3 * 1 + ii) + CC(C_UI_PIJ + 3 * 1 + ii));
                    o[T9 * npl + i] = 0.5 * sum;
                }
                /* pressure spatial flux (2/rho)<dp dv>, rho = 1 */
                o[T10 * npl + i] = 2.0 * (PR(P_PV, j1) + PR(P_PV, j2) - CC(C_PV) - CC(C_VP));
                /* production: -2<du dv> (dU/dy)* and -2<du v*> d(dU/dy) */
                double dudv = PR(P_UV, j1) + PR(P_UV, j2) - CC(C_UV) - CC(C_VU);
                double duvs = 0.5 * (PR(P_UV, j2) - PR(P_UV, j1) + CC(C_VU) - CC(C_UV));
                o[T12 * npl + i] = -2.0 * dudv * Sstar;
                o[T13 * npl + i] = -2.0 * duvs * dS;
                /* dissipation -4<eps*> */
                o[T14 * npl + i] = -2.0 * (PR(P_EPS, j1) + PR(P_EPS, j2));
#undef CC
            }
#undef PR
            /* viscous scale fluxes -2 nu d<du^2>/drx, -2 nu d<du^2>/drz: spectral in r */
            for (int dir = 0; dir < 2; ++dir) {
                for (long i = 0; i < npl; ++i) tmp[i] = o[T1 * npl + i] / (double)npl;
                fft2(nx, nz, tmp, -1, buf);
                for (int z = 0; z < nz; ++z)
                    for (int x = 0; x < nx; ++x) {
                        double kk = dir == 0 ? kx_mult(x, nx, lx) : kx_mult(z, nz, lz);
                        tmp[(long)z * nx + x] *= I * kk;
                    }
                fft2(nx, nz, tmp, +1, buf);
                double *dst = o + (dir == 0 ? T4 : T8) * npl;
                for (long i = 0; i < npl; ++i) dst[i] = -2.0 * nu * creal(tmp[i]);
            }
        }
        free(buf); free(C); free(tmp);
    }
    free(acc); free(slot); free(plane_of);
    return 0;
}
