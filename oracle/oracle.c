/*
 * FP64 CPU oracle for the biasing-force path of PySAGES (arXiv 2301.04835).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares no
 * source, header, table or helper with the HIP implementation, and the HIP
 * implementation never calls it.
 *
 * Every routine is the plain definition of the quantity it returns, written
 * out in double precision with sums taken sequentially in index order.  No
 * blocking, fusion or reordering is applied beyond what the definitions say.
 *
 * Units: nm, rad, kJ/mol, K.  Boltzmann constant k_B = R/1000 (CODATA 2018).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ----------------------------------------------------------------------- */
/* small vector helpers (local to the oracle)                               */
/* ----------------------------------------------------------------------- */
static void v_sub(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}
static void v_cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double v_dot(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

double orc_kB(void) { return 0.008314462618; }

/* ----------------------------------------------------------------------- */
/* O1  Dihedral angle of four points (FourPointCV / DihedralAngle, the CV   */
/*     list of Sec. 2.2) and its gradient.                                  */
/*                                                                          */
/*   b1 = r2-r1, b2 = r3-r2, b3 = r4-r3, n1 = b1 x b2, n2 = b2 x b3,         */
/*   phi = atan2(|b2| b1.n2, n1.n2)  in (-pi, pi].                           */
/*   Gradient: Blondel & Karplus, J. Comput. Chem. 17 (1996) 1132.          */
/* ----------------------------------------------------------------------- */
int orc_dihedral(const double *r /* 4x3 */, double *phi, double *grad /* 4x3 or NULL */)
{
    double b1[3], b2[3], b3[3], n1[3], n2[3];
    v_sub(r + 3, r + 0, b1);
    v_sub(r + 6, r + 3, b2);
    v_sub(r + 9, r + 6, b3);
    v_cross(b1, b2, n1);
    v_cross(b2, b3, n2);
    double lb2 = sqrt(v_dot(b2, b2));
    *phi = atan2(lb2 * v_dot(b1, n2), v_dot(n1, n2));
    if (grad) {
        double n1s = v_dot(n1, n1), n2s = v_dot(n2, n2), b2s = lb2 * lb2;
        if (n1s == 0.0 || n2s == 0.0 || b2s == 0.0) return 1; /* undefined */
        double p = v_dot(b1, b2) / b2s;
        double q = v_dot(b3, b2) / b2s;
        for (int k = 0; k < 3; ++k) {
            double g1 = -lb2 / n1s * n1[k];
            double g4 = lb2 / n2s * n2[k];
            grad[0 + k] = g1;
            grad[3 + k] = -(1.0 + p) * g1 + q * g4;
            grad[6 + k] = p * g1 - (1.0 + q) * g4;
            grad[9 + k] = g4;
        }
    }
    return 0;
}

/* ----------------------------------------------------------------------- */
/* O2  Radius of gyration (RadiusofGyration, CV list of Sec. 2.2),          */
/*     unweighted: Rg = sqrt( (1/N) sum_i |r_i - rbar|^2 ),                  */
/*     dRg/dr_i = (r_i - rbar) / (N Rg).                                     */
/* ----------------------------------------------------------------------- */
int orc_gyration(const double *pos /* n x 3 */, int64_t n, double *rg, double *grad /* n x 3 or NULL */)
{
    if (n <= 0) return 1;
    double c[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) c[k] += pos[3 * i + k];
    for (int k = 0; k < 3; ++k) c[k] /= (double)n;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            double d = pos[3 * i + k] - c[k];
            s += d * d;
        }
    *rg = sqrt(s / (double)n);
    if (grad) {
        if (*rg == 0.0) return 1;
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) grad[3 * i + k] = (pos[3 * i + k] - c[k]) / ((double)n * *rg);
    }
    return 0;
}

/* ----------------------------------------------------------------------- */
/* O3  Rational switching function of a coordination number (the form used */
/*     by PLUMED, which the paper cites):                                   */
/*        s(r) = (1 - x^n) / (1 - x^m),  x = r / r0.                          */
/*     Dividing numerator and denominator by (1 - x) removes the removable   */
/*     singularity at x = 1 exactly:  s = P_n(x) / P_m(x),  P_k = sum_{i<k} x^i, */
/*     so s(r0) = n/m with no special case and no cancellation near r0.     */
/*     ds/dr = (P_n' P_m - P_n P_m') / (P_m^2 r0).                             */
/* ----------------------------------------------------------------------- */
static void poly_geo(double x, int k, double *p, double *dp)
{
    double s = 0.0, ds = 0.0, xi = 1.0; /* xi = x^i */
    for (int i = 0; i < k; ++i) {
        s += xi;
        if (i + 1 < k) ds += (double)(i + 1) * xi; /* d/dx x^(i+1) = (i+1) x^i */
        xi *= x;
    }
    *p = s;
    *dp = ds;
}

void orc_switch(double r, double r0, int n, int m, double *s, double *ds_dr)
{
    double x = r / r0, pn, dpn, pm, dpm;
    poly_geo(x, n, &pn, &dpn);
    poly_geo(x, m, &pm, &dpm);
    *s = pn / pm;
    *ds_dr = (dpn * pm - pn * dpm) / (pm * pm) / r0;
}

/* minimum-image displacement a-b in an orthorhombic box (L[k] <= 0: open) */
static void min_image(const double *a, const double *b, const double *L, double *d)
{
    for (int k = 0; k < 3; ++k) {
        d[k] = a[k] - b[k];
        if (L && L[k] > 0.0) d[k] -= L[k] * rint(d[k] / L[k]);
    }
}

/*
 * Coordination number between groups A and B:
 *   CN = sum_{i in A} sum_{j in B, j != i} s(r_ij)    [ / |A| if normalize ]
 * All pairs are visited (brute force).  With rcut > 0, pairs at r >= rcut
 * contribute nothing (hard cut).  grad has natoms x 3 entries and receives
 * dCN/dr for every atom (zero for atoms in neither group).
 */
int orc_coordination(const double *pos, int64_t natoms, const int32_t *a, int64_t na, const int32_t *b,
                     int64_t nb, double r0, int n, int m, double rcut, const double *L, int normalize,
                     double *cn, double *grad)
{
    if (grad) memset(grad, 0, sizeof(double) * 3 * (size_t)natoms);
    double total = 0.0;
    double scale = normalize ? 1.0 / (double)na : 1.0;
    for (int64_t ii = 0; ii < na; ++ii) {
        int32_t i = a[ii];
        for (int64_t jj = 0; jj < nb; ++jj) {
            int32_t j = b[jj];
            if (i == j) continue;
            double d[3];
            min_image(pos + 3 * (size_t)i, pos + 3 * (size_t)j, L, d);
            double r = sqrt(v_dot(d, d));
            if (rcut > 0.0 && r >= rcut) continue;
            double s, ds;
            orc_switch(r, r0, n, m, &s, &ds);
            total += s;
            if (grad && r > 0.0) {
                for (int k = 0; k < 3; ++k) {
                    double g = scale * ds * d[k] / r;
                    grad[3 * (size_t)i + k] += g;
                    grad[3 * (size_t)j + k] -= g;
                }
            }
        }
    }
    *cn = total * scale;
    (void)natoms;
    return 0;
}

/* ----------------------------------------------------------------------- */
/* O4  Sum of Gaussian hills (metadynamics, Sec. 2.1.5):                    */
/*   D_kd = xi_d - s_kd, wrapped to the minimum image for periodic CVs      */
/*   g_k  = exp( -sum_d D_kd^2 / (2 sigma_d^2) )                            */
/*   V    = sum_k h_k g_k,   dV/dxi_d = -sum_k h_k g_k D_kd / sigma_d^2      */
/* period[d] > 0 marks CV d periodic with that period.                      */
/* ----------------------------------------------------------------------- */
void orc_hillsum(int D, const double *xi, int64_t K, const double *centers /* K x D */,
                 const double *heights, const double *sigma, const double *period, double *V,
                 double *dV /* D or NULL */)
{
    double v = 0.0;
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t k = 0; k < K; ++k) {
        double q = 0.0, dl[8];
        for (int d = 0; d < D; ++d) {
            double x = xi[d] - centers[(size_t)k * D + d];
            if (period && period[d] > 0.0) x -= period[d] * rint(x / period[d]);
            dl[d] = x;
            q += x * x / (2.0 * sigma[d] * sigma[d]);
        }
        double e = heights[k] * exp(-q);
        v += e;
        for (int d = 0; d < D; ++d) g[d] += e * dl[d];
    }
    *V = v;
    if (dV)
        for (int d = 0; d < D; ++d) dV[d] = -g[d] / (sigma[d] * sigma[d]);
}

/*
 * Hill sums for a batch of walkers (replicas, Sec. 2 on parallel runs).
 * Walker w owns hills [hill_off[w], hill_off[w+1]); with hill_off == NULL
 * every walker uses all K hills (a shared bias).  nthreads > 1 spreads the
 * walkers over OpenMP threads; each walker's sum is still sequential.
 */
void orc_hillsum_batch(int W, int D, const double *xi /* W x D */, const int64_t *hill_off, int64_t K,
                       const double *centers, const double *heights, const double *sigma,
                       const double *period, double *V /* W */, double *dV /* W x D */, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int w = 0; w < W; ++w) {
        int64_t k0 = hill_off ? hill_off[w] : 0;
        int64_t k1 = hill_off ? hill_off[w + 1] : K;
        orc_hillsum(D, xi + (size_t)w * D, k1 - k0, centers + (size_t)k0 * D, heights + k0, sigma, period,
                    V + w, dV ? dV + (size_t)w * D : NULL);
    }
#ifndef _OPENMP
    (void)nthreads;
#endif
}

/* ----------------------------------------------------------------------- */
/* O5  Well-tempered height law (Barducci et al. 2008; Sec. 2.1.5):         */
/*       h = w exp( -V(s) / (k_B dT) ),  dT = (gamma - 1) T                   */
/* The sequence below deposits K hills one after another at the given       */
/* centres, each height using the bias of the hills deposited before it.    */
/* round_f32 != 0 stores every height rounded to binary32 before it enters  */
/* later sums (the storage precision of a hill list kept in single).        */
/* kdT <= 0 means plain metadynamics (constant height w).                   */
/* ----------------------------------------------------------------------- */
double orc_wt_height(double w, double V, double kdT)
{
    if (!(kdT > 0.0) || isinf(kdT)) return w;
    return w * exp(-V / kdT);
}

void orc_wt_sequence(int D, int64_t K, const double *centers, double w, double kdT, const double *sigma,
                     const double *period, int round_f32, double *heights /* out, K */)
{
    for (int64_t k = 0; k < K; ++k) {
        double V;
        orc_hillsum(D, centers + (size_t)k * D, k, centers, heights, sigma, period, &V, NULL);
        double h = orc_wt_height(w, V, kdT);
        heights[k] = round_f32 ? (double)(float)h : h;
    }
}
