/*
 * hsd_oracle.c -- plain FP64 CPU oracle for the H^-s surface distance.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP library.
 *
 * Convention (the reading of Section 2 used throughout): the transform of a
 * measure is  mu^(xi) = \int exp(-i xi.x) dmu(x)  (no 2*pi in the exponent).
 *
 * What is computed, each function citing the passage it follows:
 *
 *  - oracle_tri_ft: the exact transform of one flat triangle, eq.
 *    (simplex32_ft) of Section 2.2 moved to the exp(-i xi.x) convention.  The
 *    closed form there is the second divided difference of exp at the three
 *    points z_j = -i xi.v_j, times the area ratio gamma = |e1 x e2|
 *    (Hermite-Genocchi).  It is evaluated with the three phases sorted and
 *    rearranged through first differences (exp(-i*mid)*sinc(half gap)) so no
 *    quotient of two small numbers appears; when the largest phase gap is
 *    below tau it uses the power series of the divided difference instead
 *    (the cancellation Section 3.1 warns about for nearly degenerate
 *    triangles or xi nearly orthogonal to an edge).
 *  - oracle_transform: mu_h^(xi_k) = sum over triangles (linearity of the
 *    transform, Section 3.1), Neumaier-compensated in triangle order.
 *  - oracle_point_sum: sum_j c_j exp(-i xi_k.x_j), the exponential sum of a
 *    weighted Dirac point cloud (eqs. change_variable_approx and
 *    def_nufft_type1) evaluated directly.
 *  - oracle_grad: d(d^2)/dv by forward-mode dual numbers (9 directions: the
 *    three vertices of one triangle) pushed through the same evaluation as
 *    oracle_tri_ft, contracted with the per-node coefficients 2 W_k conj(R_k).
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#define ND 9 /* derivative directions: 3 vertices x 3 coordinates */

/* ------------------------------------------------------------------ */
/* real scalar helpers                                                 */
/* ------------------------------------------------------------------ */

/* sin(x)/x, with its Maclaurin series near 0 */
static double sinc_v(double x)
{
    if (fabs(x) < 0.05) {
        double x2 = x * x;
        return 1.0 - x2 / 6.0 + x2 * x2 / 120.0 - x2 * x2 * x2 / 5040.0 +
               x2 * x2 * x2 * x2 / 362880.0;
    }
    return sin(x) / x;
}
/* d/dx sin(x)/x */
static double sinc_d(double x)
{
    if (fabs(x) < 0.05) {
        double x2 = x * x;
        return x * (-1.0 / 3.0 + x2 / 30.0 - x2 * x2 / 840.0 + x2 * x2 * x2 / 45360.0);
    }
    return (cos(x) - sin(x) / x) / x;
}
/* (1 - cos x)/x = 2 sin^2(x/2)/x, with its series near 0 */
static double cosc_v(double x)
{
    if (fabs(x) < 0.05) {
        double x2 = x * x;
        return x * (0.5 - x2 / 24.0 + x2 * x2 / 720.0 - x2 * x2 * x2 / 40320.0);
    }
    double s = sin(0.5 * x);
    return 2.0 * s * s / x;
}
/* d/dx (1 - cos x)/x = (sin x - (1-cos x)/x)/x */
static double cosc_d(double x)
{
    if (fabs(x) < 0.05) {
        double x2 = x * x;
        return 0.5 - x2 / 8.0 + x2 * x2 / 144.0 - x2 * x2 * x2 / 5760.0;
    }
    return (sin(x) - cosc_v(x)) / x;
}

/* ------------------------------------------------------------------ */
/* dual numbers: value + ND partial derivatives                        */
/* ------------------------------------------------------------------ */
typedef struct { double v; double d[ND]; } dual;

static dual dconst(double c) { dual r; r.v = c; memset(r.d, 0, sizeof r.d); return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * s; return r; }
static dual ddiv(dual a, dual b)
{
    dual r; r.v = a.v / b.v;
    for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}
static dual dsqrt(dual a)
{
    dual r; r.v = sqrt(a.v);
    for (int i = 0; i < ND; ++i) r.d[i] = (r.v > 0.0) ? a.d[i] / (2.0 * r.v) : 0.0;
    return r;
}
static dual dfun(dual a, double val, double der)
{
    dual r; r.v = val; for (int i = 0; i < ND; ++i) r.d[i] = der * a.d[i]; return r;
}
static dual dsin(dual a) { return dfun(a, sin(a.v), cos(a.v)); }
static dual dcos(dual a) { return dfun(a, cos(a.v), -sin(a.v)); }
static dual dsinc(dual a) { return dfun(a, sinc_v(a.v), sinc_d(a.v)); }
static dual dcosc(dual a) { return dfun(a, cosc_v(a.v), cosc_d(a.v)); }

typedef struct { dual re, im; } dcplx;

static dcplx cmul(dcplx a, dcplx b)
{
    dcplx r;
    r.re = dsub(dmul(a.re, b.re), dmul(a.im, b.im));
    r.im = dadd(dmul(a.re, b.im), dmul(a.im, b.re));
    return r;
}

/* Number of series terms of the divided difference used below tau. */
#define TAYLOR_NMAX 10

/*
 * Exact transform of the triangle (p[0],p[1],p[2]) at frequency xi, as a dual
 * number in the 9 vertex coordinates (seeded by the caller).  Steps:
 *   J = |e1 x e2| (gamma of eq. simplex32_ft, the area ratio to the standard
 *   simplex);  theta_j = xi.p_j, with the two offsets theta_j - theta_0 taken
 *   from the edge dot products;  sort the offsets; a, b = the two consecutive
 *   gaps, G = a + b;
 *   G >= tau :  E = exp(-i theta_mid) (Y + i X)/G,
 *               X = sinc(b) - sinc(a),  Y = (1-cos b)/b + (1-cos a)/a;
 *   G <  tau :  E = exp(-i theta_mid) sum_n (-i)^n H_n/(n+2)!,
 *               H_n = sum_{m=0..n} (-a)^m b^(n-m);
 *   result J*E.
 */
static dcplx tri_ft_dual(const dual p[3][3], const double xi[3], double tau)
{
    dual e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = dsub(p[1][c], p[0][c]); e2[c] = dsub(p[2][c], p[0][c]); }
    dual cr[3];
    cr[0] = dsub(dmul(e1[1], e2[2]), dmul(e1[2], e2[1]));
    cr[1] = dsub(dmul(e1[2], e2[0]), dmul(e1[0], e2[2]));
    cr[2] = dsub(dmul(e1[0], e2[1]), dmul(e1[1], e2[0]));
    dual J = dsqrt(dadd(dadd(dmul(cr[0], cr[0]), dmul(cr[1], cr[1])), dmul(cr[2], cr[2])));

    dual t0 = dconst(0.0), s1 = dconst(0.0), s2 = dconst(0.0);
    for (int c = 0; c < 3; ++c) {
        t0 = dadd(t0, dscale(p[0][c], xi[c]));
        s1 = dadd(s1, dscale(e1[c], xi[c]));
        s2 = dadd(s2, dscale(e2[c], xi[c]));
    }
    dual s[3] = { dconst(0.0), s1, s2 };
    /* insertion sort of three values by .v */
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && s[j - 1].v > s[j].v; --j) { dual t = s[j]; s[j] = s[j - 1]; s[j - 1] = t; }
    dual a = dsub(s[1], s[0]);
    dual b = dsub(s[2], s[1]);
    dual G = dadd(a, b);
    dual thm = dadd(t0, s[1]);

    dcplx ph;                       /* exp(-i theta_mid) */
    ph.re = dcos(thm);
    ph.im = dscale(dsin(thm), -1.0);

    dcplx F;
    if (G.v >= tau) {
        dual X = dsub(dsinc(b), dsinc(a));
        dual Y = dadd(dcosc(b), dcosc(a));
        F.re = ddiv(Y, G);
        F.im = ddiv(X, G);
    } else {
        dual na = dscale(a, -1.0);
        dual sre = dconst(0.0), sim = dconst(0.0);
        dual pw_a = dconst(1.0);   /* (-a)^n */
        dual H = dconst(1.0);      /* H_0 */
        double fact = 2.0;         /* (n+2)! at n=0 */
        for (int n = 0; n <= TAYLOR_NMAX; ++n) {
            if (n > 0) {
                pw_a = dmul(pw_a, na);
                H = dadd(dmul(H, b), pw_a);
                fact *= (double)(n + 2);
            }
            dual term = dscale(H, 1.0 / fact);
            /* (-i)^n cycles 1, -i, -1, i */
            switch (n & 3) {
            case 0: sre = dadd(sre, term); break;
            case 1: sim = dsub(sim, term); break;
            case 2: sre = dsub(sre, term); break;
            default: sim = dadd(sim, term); break;
            }
        }
        F.re = sre;
        F.im = sim;
    }
    dcplx E = cmul(ph, F);
    dcplx out;
    out.re = dmul(J, E.re);
    out.im = dmul(J, E.im);
    return out;
}

/* Value-only version of tri_ft_dual: the same steps in plain doubles. */
static void tri_ft_value(const double *v0, const double *v1, const double *v2,
                         const double xi[3], double tau, double *re, double *im)
{
    double e1[3], e2[3], cr[3];
    for (int c = 0; c < 3; ++c) { e1[c] = v1[c] - v0[c]; e2[c] = v2[c] - v0[c]; }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double J = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double t0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int c = 0; c < 3; ++c) { t0 += xi[c] * v0[c]; s1 += xi[c] * e1[c]; s2 += xi[c] * e2[c]; }
    double s[3] = { 0.0, s1, s2 };
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && s[j - 1] > s[j]; --j) { double t = s[j]; s[j] = s[j - 1]; s[j - 1] = t; }
    double a = s[1] - s[0], b = s[2] - s[1], G = a + b, thm = t0 + s[1];
    double pr = cos(thm), pi = -sin(thm);
    double fr, fi;
    if (G >= tau) {
        double X = sinc_v(b) - sinc_v(a);
        double Y = cosc_v(b) + cosc_v(a);
        fr = Y / G;
        fi = X / G;
    } else {
        double sre = 0.0, sim = 0.0, pw_a = 1.0, H = 1.0, fact = 2.0;
        for (int n = 0; n <= TAYLOR_NMAX; ++n) {
            if (n > 0) {
                pw_a *= -a;
                H = H * b + pw_a;
                fact *= (double)(n + 2);
            }
            double term = H / fact;
            switch (n & 3) {
            case 0: sre += term; break;
            case 1: sim -= term; break;
            case 2: sre -= term; break;
            default: sim += term; break;
            }
        }
        fr = sre;
        fi = sim;
    }
    *re = J * (pr * fr - pi * fi);
    *im = J * (pr * fi + pi * fr);
}

/* Neumaier compensated accumulator */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nget(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* exported API                                                        */
/* ------------------------------------------------------------------ */

/* Single triangle transform (for unit tests). */
void oracle_tri_ft(const double *v0, const double *v1, const double *v2,
                   const double *xi, double tau, double *out /*2*/)
{
    tri_ft_value(v0, v1, v2, xi, tau, &out[0], &out[1]);
}

/*
 * mu_h^(xi_k) = sum_T sign_T * mu_T^(xi_k) for k < nn.
 * verts[nv*3], tris[nt*3] (int32), sign[nt] (NULL => all +1),
 * nodes[nn*3], out[nn*2] (re, im).  Parallel over nodes; each node sums its
 * triangles in index order with Neumaier compensation, so the result does
 * not depend on the thread count.
 */
void oracle_transform(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                      const double *sign, const double *nodes, int64_t nn,
                      double tau, double *out)
{
    (void)nv;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nn; ++k) {
        nsum sr = { 0, 0 }, si = { 0, 0 };
        const double *xi = nodes + 3 * k;
        for (int64_t t = 0; t < nt; ++t) {
            double re, im;
            tri_ft_value(verts + 3 * (int64_t)tris[3 * t], verts + 3 * (int64_t)tris[3 * t + 1],
                         verts + 3 * (int64_t)tris[3 * t + 2], xi, tau, &re, &im);
            double sg = sign ? sign[t] : 1.0;
            nadd(&sr, sg * re);
            nadd(&si, sg * im);
        }
        out[2 * k] = nget(&sr);
        out[2 * k + 1] = nget(&si);
    }
}

/*
 * Direct exponential sum of a weighted point cloud:
 *   out_k = sum_j c_j exp(-i xi_k . x_j),  c_j real.
 */
void oracle_point_sum(const double *pts, const double *c, int64_t np,
                      const double *nodes, int64_t nn, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nn; ++k) {
        nsum sr = { 0, 0 }, si = { 0, 0 };
        const double *xi = nodes + 3 * k;
        for (int64_t j = 0; j < np; ++j) {
            const double *x = pts + 3 * j;
            double th = xi[0] * x[0] + xi[1] * x[1] + xi[2] * x[2];
            nadd(&sr, c[j] * cos(th));
            nadd(&si, -c[j] * sin(th));
        }
        out[2 * k] = nget(&sr);
        out[2 * k + 1] = nget(&si);
    }
}

/*
 * Gradient contraction.  coef[nn*2] holds the complex per-node coefficients
 * q_k = 2 W_k conj(R_k); the result is
 *   grad[v] = sum_k Re( q_k * d mu_h^(xi_k) / d v )      (grad[nv*3])
 * accumulated per triangle (parallel over triangles, nodes in order), then
 * scattered to the vertices serially in triangle order.
 */
void oracle_grad(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                 const double *sign, const double *nodes, const double *coef,
                 int64_t nn, double tau, double *grad)
{
    double *tg = (double *)calloc((size_t)nt * ND, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        dual p[3][3];
        for (int j = 0; j < 3; ++j) {
            const double *vv = verts + 3 * (int64_t)tris[3 * t + j];
            for (int c = 0; c < 3; ++c) {
                p[j][c] = dconst(vv[c]);
                p[j][c].d[3 * j + c] = 1.0;
            }
        }
        nsum acc[ND];
        memset(acc, 0, sizeof acc);
        double sg = sign ? sign[t] : 1.0;
        for (int64_t k = 0; k < nn; ++k) {
            dcplx m = tri_ft_dual(p, nodes + 3 * k, tau);
            double qr = coef[2 * k], qi = coef[2 * k + 1];
            for (int i = 0; i < ND; ++i)
                nadd(&acc[i], sg * (qr * m.re.d[i] - qi * m.im.d[i]));
        }
        for (int i = 0; i < ND; ++i) tg[t * ND + i] = nget(&acc[i]);
    }
    memset(grad, 0, sizeof(double) * (size_t)nv * 3);
    for (int64_t t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j)
            for (int c = 0; c < 3; ++c)
                grad[3 * (int64_t)tris[3 * t + j] + c] += tg[t * ND + 3 * j + c];
    free(tg);
}

/* Per-triangle, per-node derivative of one triangle's transform (9 complex),
 * for unit tests of the identities. out[ND*2]. */
void oracle_tri_ft_grad(const double *v0, const double *v1, const double *v2,
                        const double *xi, double tau, double *val /*2*/, double *out)
{
    dual p[3][3];
    const double *vv[3] = { v0, v1, v2 };
    for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) {
            p[j][c] = dconst(vv[j][c]);
            p[j][c].d[3 * j + c] = 1.0;
        }
    dcplx r = tri_ft_dual(p, xi, tau);
    val[0] = r.re.v;
    val[1] = r.im.v;
    for (int i = 0; i < ND; ++i) { out[2 * i] = r.re.d[i]; out[2 * i + 1] = r.im.d[i]; }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
