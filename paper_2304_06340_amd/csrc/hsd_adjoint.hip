// hsd_adjoint.hip -- gradient of d^2 with respect to the vertices of mu.
//
// With mu_T = J_T E_T, E_T = e[z0, z1, z2] (second divided difference of exp
// at z_j = -i theta_j, theta_j = xi.v_j) and R_k = mu_h^(xi_k) - nu^(xi_k):
//
//   d(d^2)/dv_j(T) = sum_k 2 W_k Re( conj(R_k) dmu_T(xi_k)/dv_j )
//                  = a_j S_E + J V_j,
//   S_E = sum_k Re(q_k E_T(xi_k)),  V_j = sum_k Re(q_k D_j(xi_k)) xi_k,
//
// q_k = 2 W_k conj(R_k), a_j = dJ/dv_j = n_T x (v_{j+2} - v_{j+1}) and
// D_j = dE/dtheta_j.  In the sorted frame E = exp(-i theta_mid) F(a, b) with
// a = theta_mid - theta_lo, b = theta_hi - theta_mid:
//   D_lo = -exp(-i theta_mid) F_a,  D_hi = exp(-i theta_mid) F_b,
//   D_mid = -i E - D_lo - D_hi        (translation: sum_j D_j = -i E).
// F, F_a, F_b come from the closed form (Y + iX)/G and its derivatives for
// G >= tau, with series for sin(x)/x and (1-cos x)/x derivatives at small
// arguments, and from the power series of the divided difference below tau.
//
// Work split: a lane owns one triangle; the 64 lanes of a wave walk the same
// nodes (wave-uniform index, scalar loads of the direction, radius and
// q_k); grid.y splits the directions.  Per-triangle partial sums [S][nt][10]
// are combined in fixed order, turned into per-triangle vertex gradients,
// and gathered to vertices through a vertex -> (triangle, slot) CSR in fixed
// order.  No floating-point atomics.
#include "hsd_internal.hpp"
#include "hsd_math.hpp"

namespace hsd {

constexpr int kAdjNV = 10;   // S_E, V_0[3], V_1[3], V_2[3]
// Gaps are floored here (per unit radius, or per pair) so that a zero gap
// needs no special case; r times the floor stays a normal number.
constexpr double kAdjGapFloor = 1e-150;

// Maclaurin coefficients of the two derivatives:
//   d/dx sin(x)/x       = sum_{k>=1} (-1)^k     2k     x^(2k-1) / (2k+1)!
//   d/dx (1 - cos x)/x  = sum_{k>=1} (-1)^(k+1) (2k-1) x^(2k-2) / (2k)!
constexpr double dsinc_coef(int k) { return ((k & 1) ? -1.0 : 1.0) * 2.0 * k * inv_factorial(2 * k + 1); }
constexpr double dcosc_coef(int k) { return ((k & 1) ? 1.0 : -1.0) * (2.0 * k - 1.0) * inv_factorial(2 * k); }

// d/dx sin(x)/x and d/dx (1-cos x)/x (x >= 0, ix = 1/x), with the series
// (k <= 7, first omitted terms far below 1e-16 relative to the leading x/3
// and 1/2) below 0.005.  Above it the closed forms (cos x - sinc x)/x and
// (sin x - (1-cos x)/x)/x lose at most about 6 eps / x^2 to cancellation
// (2.6e-11 relative at x = 0.005, against the 1e-9 the gradient is held
// to); the low threshold makes the lanes of a wave (different triangles)
// take the series rarely: at 0.05 some lane took it in most iterations.
HSD_HD void dsinc_dcosc(double x, double ix, double sx, double cx, double sinc, double cosc, double &dsinc,
                        double &dcosc)
{
    if (x < 0.005) {
        const double x2 = x * x;
        double ps = dsinc_coef(7), pc = dcosc_coef(7);
#pragma unroll
        for (int k = 6; k >= 1; --k) {
            ps = __builtin_fma(ps, x2, dsinc_coef(k));
            pc = __builtin_fma(pc, x2, dcosc_coef(k));
        }
        dsinc = ps * x;
        dcosc = pc;
    } else {
        dsinc = (cx - sinc) * ix;
        dcosc = (sx - cosc) * ix;
    }
}

// F(a,b) = sum_n (-i)^n H_n/(n+2)! and its a- and b-derivatives, with
// H_n = b H_{n-1} + (-a)^n, dH_n/da = b dH_{n-1}/da - n (-a)^{n-1},
// dH_n/db = H_{n-1} + b dH_{n-1}/db.  Terms up to n = 9: for a + b < 0.05
// the first omitted ones are below 1e-17 relative (F: G^10 / 12!; F_a, F_b:
// 10 G^9 / 12! against the leading 1/6).
HSD_HD void dd2_series_grad(double a, double b, double F[2], double Fa[2], double Fb[2])
{
    double H = 1.0, A = 0.0, B = 0.0, pw = 1.0;   // (-a)^n
    double fr = 0.5, fi = 0.0, ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
#pragma unroll
    for (int n = 1; n <= 9; ++n) {
        const double pw_prev = pw;
        pw *= -a;
        const double Hprev = H;
        H = b * H + pw;
        A = b * A - (double)n * pw_prev;
        B = Hprev + b * B;
        const double c = inv_factorial(n + 2);
        switch (n & 3) {   // (-i)^n = 1, -i, -1, i
        case 0: fr += H * c; ar += A * c; br += B * c; break;
        case 1: fi -= H * c; ai -= A * c; bi -= B * c; break;
        case 2: fr -= H * c; ar -= A * c; br -= B * c; break;
        default: fi += H * c; ai += A * c; bi += B * c; break;
        }
    }
    F[0] = fr; F[1] = fi;
    Fa[0] = ar; Fa[1] = ai;
    Fb[0] = br; Fb[1] = bi;
}

// The sorted-frame factors of one (triangle, node) pair from its half-gap
// phases hu = exp(-i a/2), hv = exp(-i b/2): F(a, b) and its derivatives
// F_a, F_b (complex); ia, ib, iG are 1/a, 1/b, 1/(a+b) (used only where
// a, b > 0 and G >= tau).
HSD_HD void pair_factors(double a, double b, double tau, cs64 hu, cs64 hv, double ia, double ib, double iG,
                         double F[2], double Fa[2], double Fb[2])
{
    const double G = a + b;
    if (G < tau) {
        dd2_series_grad(a, b, F, Fa, Fb);
    } else {
        const double sa = 2.0 * hu.s * hu.c, ca = hu.c * hu.c - hu.s * hu.s;
        const double sb = 2.0 * hv.s * hv.c, cb = hv.c * hv.c - hv.s * hv.s;
        // sinc and (1-cos)/x of a, b (both gaps floored at kAdjGapFloor, so
        // that a zero gap gives its limits 1 and 0 without a select)
        const double sinc_a = sa * ia;
        const double sinc_b = sb * ib;
        const double cosc_a = 2.0 * hu.s * hu.s * ia;
        const double cosc_b = 2.0 * hv.s * hv.s * ib;
        double dsa, dca, dsb, dcb;
        dsinc_dcosc(a, ia, sa, ca, sinc_a, cosc_a, dsa, dca);
        dsinc_dcosc(b, ib, sb, cb, sinc_b, cosc_b, dsb, dcb);
        F[0] = (cosc_b + cosc_a) * iG;
        F[1] = (sinc_b - sinc_a) * iG;
        Fa[0] = (dca - F[0]) * iG;
        Fa[1] = (-dsa - F[1]) * iG;
        Fb[0] = (dcb - F[0]) * iG;
        Fb[1] = (dsb - F[1]) * iG;
    }
}

// E = exp(-i theta_mid) F and the derivatives D_lo, D_mid, D_hi (complex,
// in the sorted frame) of one pair; e1 = exp(-i theta_mid) as (cos, sin).
HSD_HD void pair_grad_ph(double a, double b, double tau, cs64 hu, cs64 hv, cs64 e1, double ia, double ib,
                         double iG, double E[2], double Dlo[2], double Dmid[2], double Dhi[2])
{
    double F[2], Fa[2], Fb[2];
    pair_factors(a, b, tau, hu, hv, ia, ib, iG, F, Fa, Fb);
    const double er = e1.c, ei = -e1.s;   // exp(-i theta) = (c, -s)
    E[0] = er * F[0] - ei * F[1];
    E[1] = er * F[1] + ei * F[0];
    Dlo[0] = -(er * Fa[0] - ei * Fa[1]);
    Dlo[1] = -(er * Fa[1] + ei * Fa[0]);
    Dhi[0] = er * Fb[0] - ei * Fb[1];
    Dhi[1] = er * Fb[1] + ei * Fb[0];
    // -i E = (E_im, -E_re)
    Dmid[0] = E[1] - Dlo[0] - Dhi[0];
    Dmid[1] = -E[0] - Dlo[1] - Dhi[1];
}

// Accumulate one pair into a direction's four sums from the weighted
// residual q = 2 W conj(R) and the pair's factors: with Q = q exp(-i theta),
//   S_E  += Re(q E)        = Re(Q F)
//   S_I  += r Im(q E)      = r Im(Q F)
//   u_lo += r Re(q D_lo)   = -r Re(Q F_a)
//   u_hi += r Re(q D_hi)   =  r Re(Q F_b)
// and u_mid = S_I - u_lo - u_hi once per direction (translation: the three
// derivatives sum to -i E), so E and the D_j are never formed.
HSD_HD void pair_accumulate(double qr, double qi, cs64 e1, double r, const double F[2], const double Fa[2],
                            const double Fb[2], double &sE, double &sI, double &ulo, double &uhi)
{
    // exp(-i theta) = (c, -s):  Q = (qr c + qi s) + i (qi c - qr s)
    const double Qr = __builtin_fma(qr, e1.c, qi * e1.s);
    const double Qi = __builtin_fma(qi, e1.c, -qr * e1.s);
    sE = __builtin_fma(Qr, F[0], __builtin_fma(-Qi, F[1], sE));
    const double rQr = r * Qr, rQi = r * Qi;
    sI = __builtin_fma(rQr, F[1], __builtin_fma(rQi, F[0], sI));
    ulo = __builtin_fma(-rQr, Fa[0], __builtin_fma(rQi, Fa[1], ulo));
    uhi = __builtin_fma(rQr, Fb[0], __builtin_fma(-rQi, Fb[1], uhi));
}

HSD_HD void pair_grad(double thmid, double a, double b, double tau, double E[2], double Dlo[2],
                      double Dmid[2], double Dhi[2])
{
    a = fmax(a, kAdjGapFloor);
    b = fmax(b, kAdjGapFloor);
    pair_grad_ph(a, b, tau, sincos64(0.5 * a), sincos64(0.5 * b), sincos64(thmid), 1.0 / a, 1.0 / b, 1.0 / (a + b), E,
                 Dlo, Dmid, Dhi);
}

// Per-direction scatter of the three sorted-frame sums to the vertex slots.
HSD_HD void adjoint_scatter(double nx, double ny, double nz, const double u[3], const int idx[3],
                            double acc[kAdjNV])
{
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int j = idx[p];
        // scatter by vertex index with selects (no dynamic register index)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            const double w = (j == jj) ? u[p] : 0.0;
            acc[1 + 3 * jj] += w * nx;
            acc[2 + 3 * jj] += w * ny;
            acc[3 + 3 * jj] += w * nz;
        }
    }
}

// Lane body for spherical-product rules (radial nodes m_p +- h x_k of P
// panels with n nodes each, r index = p n + j): the phases of the three
// per-(triangle, direction) constants c (theta_mid, a/2, b/2) at radius
// m_p +- h x_k are exp(-i m_p c) exp(-+i h x_k c), with the offsets' phases
// computed once per direction and the panel centres stepped by
// exp(-2 i h c), for every node (the nodes h - h x_k of panel 0 included:
// their half-gap sines then carry an absolute rounding of the larger angles
// (h + h x_k) c, as in the forward kernel).  1/r comes
// from the rule's table of reciprocal radii (the same for all lanes), 1/a
// and 1/b from per-direction reciprocals.
HSD_HD void adjoint_lane_sp(const TriRec &T, const double *dirs, const double *iradii, int P, int n, double h,
                            const double *hx_tab, int64_t d_begin, int64_t d_end, const double2 *resid,
                            const double *wdir, const double *wtab, double tau, double acc[kAdjNV])
{
    const int n_rad = P * n, nh = n / 2;
    for (int i = 0; i < kAdjNV; ++i) acc[i] = 0.0;
    for (int64_t d = d_begin; d < d_end; ++d) {
        const double nx = dirs[3 * d], ny = dirs[3 * d + 1], nz = dirs[3 * d + 2];
        const double t0 = nx * T.p0[0] + ny * T.p0[1] + nz * T.p0[2];
        const double s1 = nx * T.e1[0] + ny * T.e1[1] + nz * T.e1[2];
        const double s2 = nx * T.e2[0] + ny * T.e2[1] + nz * T.e2[2];
        double v0 = 0.0, v1 = s1, v2 = s2;
        int i0 = 0, i1 = 1, i2 = 2;
        if (v1 < v0) { double t = v0; v0 = v1; v1 = t; int ti = i0; i0 = i1; i1 = ti; }
        if (v2 < v1) { double t = v1; v1 = v2; v2 = t; int ti = i1; i1 = i2; i2 = ti; }
        if (v1 < v0) { double t = v0; v0 = v1; v1 = t; int ti = i0; i0 = i1; i1 = ti; }
        const double al = fmax(v1 - v0, kAdjGapFloor), be = fmax(v2 - v1, kAdjGapFloor), tmid = t0 + v1;
        const double ial = 1.0 / al, ibe = 1.0 / be, iGc = 1.0 / (al + be);
        const double wd = wdir[d];
        const double fr[3] = {tmid, 0.5 * al, 0.5 * be};
        cs64 step[3], c0[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            c0[c] = sincos64(h * fr[c]);
            step[c] = pmul(c0[c], c0[c]);
        }
        double sE = 0.0, sI = 0.0, ulo = 0.0, uhi = 0.0;
        for (int k = 0; k < nh; ++k) {
            const double hx = hx_tab[k];
            cs64 bk[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) bk[c] = sincos64(hx * fr[c]);
            cs64 cp[3] = {c0[0], c0[1], c0[2]};
            for (int p = 0; p < P; ++p) {
                const double m = (double)(2 * p + 1) * h;
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const double r = sg == 0 ? m + hx : m - hx;
                    const int ir = p * n + (sg == 0 ? nh + k : nh - 1 - k);
                    cs64 ph[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) ph[c] = sg == 0 ? pmul(cp[c], bk[c]) : pmulc(cp[c], bk[c]);
                    const double irr = iradii[ir];
                    const int64_t node = d * n_rad + ir;
                    const double W = wd * wtab[ir];
                    const double2 R = resid[node];
                    const double qr = 2.0 * W * R.x, qi = -2.0 * W * R.y;
                    double F[2], Fa[2], Fb[2];
                    pair_factors(r * al, r * be, tau, ph[1], ph[2], irr * ial, irr * ibe, irr * iGc, F, Fa, Fb);
                    pair_accumulate(qr, qi, ph[0], r, F, Fa, Fb, sE, sI, ulo, uhi);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) cp[c] = pmul(cp[c], step[c]);
            }
        }
        acc[0] += sE;
        const double u[3] = {ulo, sI - ulo - uhi, uhi};
        const int idx[3] = {i0, i1, i2};
        adjoint_scatter(nx, ny, nz, u, idx, acc);
    }
}

// Lane body: one triangle against directions [d_begin, d_end) x all radii.
// acc[10] = (S_E, V_0, V_1, V_2) for this slice.
HSD_HD void adjoint_lane(const TriRec &T, const double *dirs, const double *radii, int n_rad,
                         int64_t d_begin, int64_t d_end, const double2 *resid, const double *wdir,
                         const double *wtab, double tau, double acc[kAdjNV])
{
    for (int i = 0; i < kAdjNV; ++i) acc[i] = 0.0;
    for (int64_t d = d_begin; d < d_end; ++d) {
        const double nx = dirs[3 * d], ny = dirs[3 * d + 1], nz = dirs[3 * d + 2];
        const double t0 = nx * T.p0[0] + ny * T.p0[1] + nz * T.p0[2];
        const double s1 = nx * T.e1[0] + ny * T.e1[1] + nz * T.e1[2];
        const double s2 = nx * T.e2[0] + ny * T.e2[1] + nz * T.e2[2];
        // sort (0, s1, s2) keeping the vertex index of each position
        double v0 = 0.0, v1 = s1, v2 = s2;
        int i0 = 0, i1 = 1, i2 = 2;
        if (v1 < v0) { double t = v0; v0 = v1; v1 = t; int ti = i0; i0 = i1; i1 = ti; }
        if (v2 < v1) { double t = v1; v1 = v2; v2 = t; int ti = i1; i1 = i2; i2 = ti; }
        if (v1 < v0) { double t = v0; v0 = v1; v1 = t; int ti = i0; i0 = i1; i1 = ti; }
        const double al = fmax(v1 - v0, kAdjGapFloor), be = fmax(v2 - v1, kAdjGapFloor), tmid = t0 + v1;
        const double wd = wdir ? wdir[d] : 1.0;
        double sE = 0.0, sI = 0.0, ulo = 0.0, uhi = 0.0;
        for (int ir = 0; ir < n_rad; ++ir) {
            const double r = radii[ir];
            const int64_t node = d * n_rad + ir;
            const double W = wd * wtab[wdir ? ir : node];
            const double2 R = resid[node];
            const double qr = 2.0 * W * R.x, qi = -2.0 * W * R.y;   // q = 2 W conj(R)
            const double a = r * al, b = r * be, G = a + b;
            double F[2], Fa[2], Fb[2];
            pair_factors(a, b, tau, sincos64(0.5 * a), sincos64(0.5 * b), 1.0 / a, 1.0 / b, 1.0 / G, F, Fa, Fb);
            pair_accumulate(qr, qi, sincos64(r * tmid), r, F, Fa, Fb, sE, sI, ulo, uhi);
        }
        acc[0] += sE;
        const double u[3] = {ulo, sI - ulo - uhi, uhi};
        const int idx[3] = {i0, i1, i2};
        adjoint_scatter(nx, ny, nz, u, idx, acc);
    }
}

// Held to 3 waves per SIMD (168 VGPRs, a few spills outside the node loop):
// about 4% faster than the 2 its 204 registers would allow; at 4 the node
// loop spills.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_adjoint(const TriRec *__restrict__ tris, int64_t nt,
                                                 const double *__restrict__ dirs, int64_t n_dir,
                                                 const double *__restrict__ radii, int n_rad,
                                                 const double2 *__restrict__ resid,
                                                 const double *__restrict__ wdir,
                                                 const double *__restrict__ wtab, double tau, int P, int n,
                                                 double h, const double *__restrict__ hx_tab,
                                                 const double *__restrict__ iradii, double *__restrict__ part)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int S = gridDim.y;
    const int64_t d_begin = n_dir * blockIdx.y / S;
    const int64_t d_end = n_dir * (blockIdx.y + 1) / S;
    const TriRec T = tris[t < nt ? t : 0];
    double acc[kAdjNV];
    if (hx_tab)   // spherical-product rule: radial product structure
        adjoint_lane_sp(T, dirs, iradii, P, n, h, hx_tab, d_begin, d_end, resid, wdir, wtab, tau, acc);
    else
        adjoint_lane(T, dirs, radii, n_rad, d_begin, d_end, resid, wdir, wtab, tau, acc);
    if (t >= nt) return;
    double *o = part + ((int64_t)blockIdx.y * nt + t) * kAdjNV;
#pragma unroll
    for (int i = 0; i < kAdjNV; ++i) o[i] = acc[i];
}

// Sum the S partials in fixed order and form g_j = a_j S_E + J V_j.
__global__ void k_adjoint_finish(const TriRec *__restrict__ tris, int64_t nt, int S,
                                 const double *__restrict__ part, double *__restrict__ tri_grad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double acc[kAdjNV];
    for (int i = 0; i < kAdjNV; ++i) acc[i] = 0.0;
    for (int s = 0; s < S; ++s)
        for (int i = 0; i < kAdjNV; ++i) acc[i] += part[((int64_t)s * nt + t) * kAdjNV + i];
    const TriRec T = tris[t];
    const double e1[3] = {T.e1[0], T.e1[1], T.e1[2]}, e2[3] = {T.e2[0], T.e2[1], T.e2[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double J = T.J;
    const double iJ = J > 0.0 ? 1.0 / J : 0.0;
    for (int c = 0; c < 3; ++c) n[c] *= iJ;
    // edges opposite each vertex: v2 - v1 = e2 - e1, v0 - v2 = -e2, v1 - v0 = e1
    const double opp[3][3] = {{e2[0] - e1[0], e2[1] - e1[1], e2[2] - e1[2]},
                              {-e2[0], -e2[1], -e2[2]},
                              {e1[0], e1[1], e1[2]}};
    for (int j = 0; j < 3; ++j) {
        const double *o = opp[j];
        const double aj[3] = {n[1] * o[2] - n[2] * o[1], n[2] * o[0] - n[0] * o[2], n[0] * o[1] - n[1] * o[0]};
        for (int c = 0; c < 3; ++c) tri_grad[t * 9 + 3 * j + c] = aj[c] * acc[0] + J * acc[1 + 3 * j + c];
    }
}

// grad[v] = sum over CSR entries (3 t + slot), increasing t.
__global__ void k_gather(int64_t nv, const int32_t *__restrict__ ptr, const int32_t *__restrict__ ent,
                         const double *__restrict__ tri_grad, double *__restrict__ grad)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) {
        const int64_t ts = ent[e];   // 3 t + slot
        const int64_t t = ts / 3, j = ts - 3 * t;
        g0 += tri_grad[t * 9 + 3 * j];
        g1 += tri_grad[t * 9 + 3 * j + 1];
        g2 += tri_grad[t * 9 + 3 * j + 2];
    }
    grad[3 * v] = g0;
    grad[3 * v + 1] = g1;
    grad[3 * v + 2] = g2;
}

int adjoint_splits(int64_t nt, int64_t n_dir, int num_cu)
{
    const int64_t waves = ((nt + 255) / 256) * 4;
    const int64_t target = (int64_t)num_cu * 4 * 8;
    int64_t S = (target + waves - 1) / waves;
    S = std::max<int64_t>(1, std::min<int64_t>(S, n_dir));
    return (int)std::min<int64_t>(S, 65535);
}

hsd_status launch_adjoint_raw(hipStream_t st, const TriRec *tris, int64_t nt, const double *dirs, int64_t n_dir,
                              const double *radii, int n_rad, const double2 *resid, const double *wdir,
                              const double *wtab, double tau, int S, double *part, double *tri_grad, int P, int n,
                              double h, const double *hx_tab, const double *iradii)
{
    if (nt == 0) return HSD_OK;
    if (hx_tab && (P <= 0 || n <= 0 || n % 2 || P * n != n_rad || !wdir || !iradii)) {
        set_error("adjoint: inconsistent spherical-product description");
        return HSD_EINVAL;
    }
    const int64_t blocks = (nt + 255) / 256;
    hipLaunchKernelGGL(k_adjoint, dim3((unsigned)blocks, (unsigned)S), dim3(256), 0, st, tris, nt, dirs, n_dir,
                       radii, n_rad, resid, wdir, wtab, tau, P, n, h, hx_tab, iradii, part);
    HSD_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_adjoint_finish, dim3((unsigned)blocks), dim3(256), 0, st, tris, nt, S, part, tri_grad);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

hsd_status launch_gather(hipStream_t st, const hsd_mesh *m, const double *tri_grad, double *grad)
{
    if (m->nv == 0) return HSD_OK;
    const int64_t blocks = (m->nv + 255) / 256;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, st, m->nv, m->csr_ptr.as<const int32_t>(),
                       m->csr_ent.as<const int32_t>(), tri_grad, grad);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

} // namespace hsd

#ifdef HSD_TEST_HOOKS
using namespace hsd;

extern "C" {

// CPU run of the adjoint lane body for one triangle (self checks only):
// acc[10] = (S_E, V_0, V_1, V_2) over all nodes.
void hsd__host_adjoint_lane(const double *p0, const double *e1, const double *e2, double J, const double *dirs,
                            int64_t n_dir, const double *radii, int n_rad, const double *resid,
                            const double *wtab, double tau, double *acc)
{
    TriRec T;
    for (int c = 0; c < 3; ++c) { T.p0[c] = p0[c]; T.e1[c] = e1[c]; T.e2[c] = e2[c]; }
    T.J = J;
    adjoint_lane(T, dirs, radii, n_rad, 0, n_dir, (const double2 *)resid, nullptr, wtab, tau, acc);
}

// CPU run of both adjoint lane bodies for one triangle on a spherical-product
// rule (self checks only): acc_sp from the radial product structure, acc_ref
// from per-node sin/cos; resid [n_dir * P * n] complex, wdir [n_dir],
// wtab [P * n] (radial), hx_tab [n / 2].
void hsd__host_adjoint_lane_sp(const double *p0, const double *e1, const double *e2, double J, const double *dirs,
                               int64_t n_dir, const double *radii, int P, int n, double h, const double *hx_tab,
                               const double *resid, const double *wdir, const double *wtab, double tau,
                               double *acc_sp, double *acc_ref)
{
    TriRec T;
    for (int c = 0; c < 3; ++c) { T.p0[c] = p0[c]; T.e1[c] = e1[c]; T.e2[c] = e2[c]; }
    T.J = J;
    std::vector<double> iradii((size_t)P * n);
    for (size_t i = 0; i < iradii.size(); ++i) iradii[i] = 1.0 / radii[i];
    adjoint_lane_sp(T, dirs, iradii.data(), P, n, h, hx_tab, 0, n_dir, (const double2 *)resid, wdir, wtab, tau,
                    acc_sp);
    adjoint_lane(T, dirs, radii, P * n, 0, n_dir, (const double2 *)resid, wdir, wtab, tau, acc_ref);
}

void hsd__host_pair_grad(double thmid, double a, double b, double tau, double *out /*8*/)
{
    pair_grad(thmid, a, b, tau, out, out + 2, out + 4, out + 6);
}

} // extern "C"
#endif // HSD_TEST_HOOKS
