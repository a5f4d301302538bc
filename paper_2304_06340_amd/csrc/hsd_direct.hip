// hsd_direct.hip -- direct-sum kernels for mu_h^(xi_k) = sum_T mu_T^(xi_k),
// the per-node finalize (residual against the target, Sobolev weight) and
// the two-level deterministic reduction to d^2.
//
// Per pair the exact triangle transform (eq. simplex32_ft, Section 2.2) is
// evaluated as J * e[z0, z1, z2], the second divided difference of exp at
// z_j = -i xi.v_j (Hermite-Genocchi).  With the three phases sorted,
// a = theta_mid - theta_lo, b = theta_hi - theta_mid, G = a + b:
//
//   G >= tau : e = exp(-i theta_mid) (Y + i X) / G,
//              X = sin(b)/b - sin(a)/a,  Y = 2 sin^2(b/2)/b + 2 sin^2(a/2)/a
//   G <  tau : e = exp(-i theta_mid) sum_n (-i)^n H_n / (n+2)!,
//              H_n = sum_m (-a)^m b^(n-m)
//
// which avoids the cancellation of the closed form for nearly degenerate
// triangles or xi nearly orthogonal to an edge (Section 3.1).
//
// Spherical-product kernel ("sp"): for a node xi = r n, every phase is r
// times a per-(triangle, direction) constant c, and the radial nodes of a
// panel are m_p +- h x_k (panel centre m_p, half width h, Gauss-Legendre
// node x_k).  So exp(-i r c) = exp(-i m_p c) exp(-+i h x_k c): one lane owns
// a direction n, a node pair +-x_k and a group of PG panels (2*PG nodes); per
// triangle it computes 2 sine/cosine pairs per constant (exp(-i h x_k c),
// exp(-i h c)), walks the panel centres with exp(-i 2h c), and spends only
// complex products per node.  All 1/r factors of the closed branch are
// deferred: the lane accumulates r^2 mu^ and divides once at the end.
//
// Triangles are read by whole wavefronts in lock step (uniform index), so
// their 80-byte records arrive through scalar loads into SGPRs; no LDS
// staging is needed.  Sums: per-lane FP64 partials over tiles of TILE
// triangles are merged into running totals (blocked summation), K triangle
// splits write [K][N] partial transforms summed in fixed order by the
// finalize kernel; no floating-point atomics anywhere.
#include <vector>

#include "hsd_internal.hpp"
#include "hsd_math.hpp"

namespace hsd {

constexpr int kTile = 32;          // triangles per blocked-summation tile
constexpr double kGapFloor = 1e-150;
// Gap floor of the mixed form: keeps 2J/(gap G) finite in FP32 (an exactly
// zero gap becomes 1e-18, changing mu_T by ~1e-18 relative).
constexpr double kGapFloor32 = 1e-18;

// ---------------------------------------------------------------------------
// Lane bodies (host+device so the library can run them on the CPU in its
// self checks; the kernels below are thin wrappers).
// ---------------------------------------------------------------------------

// Triangle gi of the concatenated list (A with sign +1, then B with -1).
HSD_HD const TriRec *tri_at(const TriRec *A, int64_t nA, const TriRec *B, int64_t gi, double &J)
{
    const bool inA = gi < nA;
    const TriRec *rp = inA ? (A + gi) : (B + (gi - nA));
    J = inA ? rp->J : -rp->J;
    return rp;
}

// Spherical-product lane, FP64: direction (nx,ny,nz), node pair +-hx, panels
// p0 .. p0+PG-1 of half width h.  Returns r^2 mu^ per slot (slot 2*pl+sg,
// sg 0: r = m_p + hx, sg 1: r = m_p - hx) summed over triangles
// [t_begin, t_end) in tiles of kTile.
template <int PG>
HSD_HD void sp_lane_f64(const TriRec *A, int64_t nA, const TriRec *B, int64_t t_begin, int64_t t_end,
                        double nx, double ny, double nz, double hx, int p0, double h, double tau,
                        double *tot_re, double *tot_im)
{
    constexpr int NS = 2 * PG;
#pragma unroll
    for (int i = 0; i < NS; ++i) { tot_re[i] = 0.0; tot_im[i] = 0.0; }
    for (int64_t t0i = t_begin; t0i < t_end; t0i += kTile) {
        double acc_re[NS], acc_im[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) { acc_re[i] = 0.0; acc_im[i] = 0.0; }
        const int64_t tile_end = (t0i + kTile < t_end) ? t0i + kTile : t_end;
        for (int64_t gi = t0i; gi < tile_end; ++gi) {
            double J;
            const TriRec *rp = tri_at(A, nA, B, gi, J);
            const double t0 = __builtin_fma(nx, rp->p0[0], __builtin_fma(ny, rp->p0[1], nz * rp->p0[2]));
            const double d1 = __builtin_fma(nx, rp->e1[0], __builtin_fma(ny, rp->e1[1], nz * rp->e1[2]));
            const double d2 = __builtin_fma(nx, rp->e2[0], __builtin_fma(ny, rp->e2[1], nz * rp->e2[2]));
            double lo, mid, hi;
            sort3(0.0, d1, d2, lo, mid, hi);
            const double ac = fmax(mid - lo, kGapFloor);
            const double bc = fmax(hi - mid, kGapFloor);
            const double tmid = t0 + mid;
            const double iG = rcp64(ac + bc);
            const double Ka = 2.0 * J * rcp64(ac) * iG;
            const double Kb = 2.0 * J * rcp64(bc) * iG;
            const double r_thr = tau * iG;
            const double fr[3] = {tmid, 0.5 * ac, 0.5 * bc};
            cs64 Bk[3], S[3], Cp[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Bk[c] = sincos64(hx * fr[c]);
                const cs64 Eh = sincos64(h * fr[c]);
                S[c] = pmul(Eh, Eh);
                Cp[c] = (p0 == 0) ? Eh : sincos64((double)(2 * p0 + 1) * h * fr[c]);
            }
#pragma unroll
            for (int pl = 0; pl < PG; ++pl) {
                const double m = (double)(2 * (p0 + pl) + 1) * h;
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const int slot = 2 * pl + sg;
                    const double r = sg == 0 ? m + hx : m - hx;
                    cs64 E1, Eu, Ev;
                    if (sg == 1 && p0 + pl == 0) {
                        // r = h - hx is small: forming its phases from
                        // exp(-i h c) exp(+i hx c) would lose relative
                        // accuracy in sin(r c), so evaluate them directly
                        E1 = sincos64(r * fr[0]);
                        Eu = sincos64(r * fr[1]);
                        Ev = sincos64(r * fr[2]);
                    } else {
                        E1 = sg == 0 ? pmul(Cp[0], Bk[0]) : pmulc(Cp[0], Bk[0]);
                        Eu = sg == 0 ? pmul(Cp[1], Bk[1]) : pmulc(Cp[1], Bk[1]);
                        Ev = sg == 0 ? pmul(Cp[2], Bk[2]) : pmulc(Cp[2], Bk[2]);
                    }
                    const double Pv = Kb * Ev.s;
                    const double Pu = Ka * Eu.s;
                    double Yr = __builtin_fma(Pv, Ev.s, Pu * Eu.s);
                    double Xr = __builtin_fma(Pv, Ev.c, -Pu * Eu.c);
                    if (r < r_thr) {
                        double fre, fim;
                        dd2_series(r * ac, r * bc, fre, fim);
                        const double r2J = r * r * J;
                        Yr = r2J * fre;
                        Xr = r2J * fim;
                    }
                    acc_re[slot] += __builtin_fma(E1.c, Yr, E1.s * Xr);
                    acc_im[slot] += __builtin_fma(E1.c, Xr, -E1.s * Yr);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) Cp[c] = pmul(Cp[c], S[c]);
            }
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) { tot_re[i] += acc_re[i]; tot_im[i] += acc_im[i]; }
    }
}

// Spherical-product lane, mixed precision: FP64 geometry, gaps, phase
// constants and their reduction mod pi/2; FP32 sin/cos of the reduced phases,
// FP32 per-node products and tile sums; FP64 running totals; series branch
// in FP64.  Same slot layout as sp_lane_f64.
template <int PG>
HSD_HD void sp_lane_mixed(const TriRec *A, int64_t nA, const TriRec *B, int64_t t_begin, int64_t t_end,
                          double nx, double ny, double nz, double hx, int p0, double h, double tau,
                          double *tot_re, double *tot_im)
{
    constexpr int NS = 2 * PG;
    float rr[NS];
#pragma unroll
    for (int pl = 0; pl < PG; ++pl) {
        const double m = (double)(2 * (p0 + pl) + 1) * h;
        rr[2 * pl] = (float)(m + hx);
        rr[2 * pl + 1] = (float)(m - hx);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) { tot_re[i] = 0.0; tot_im[i] = 0.0; }
    for (int64_t t0i = t_begin; t0i < t_end; t0i += kTile) {
        double acc_re[NS], acc_im[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) { acc_re[i] = 0.0; acc_im[i] = 0.0; }
        const int64_t tile_end = (t0i + kTile < t_end) ? t0i + kTile : t_end;
        for (int64_t gi = t0i; gi < tile_end; ++gi) {
            double J;
            const TriRec *rp = tri_at(A, nA, B, gi, J);
            const double t0 = __builtin_fma(nx, rp->p0[0], __builtin_fma(ny, rp->p0[1], nz * rp->p0[2]));
            const double d1 = __builtin_fma(nx, rp->e1[0], __builtin_fma(ny, rp->e1[1], nz * rp->e1[2]));
            const double d2 = __builtin_fma(nx, rp->e2[0], __builtin_fma(ny, rp->e2[1], nz * rp->e2[2]));
            double lo, mid, hi;
            sort3(0.0, d1, d2, lo, mid, hi);
            const double ac = fmax(mid - lo, kGapFloor32);
            const double bc = fmax(hi - mid, kGapFloor32);
            const double tmid = t0 + mid;
            const double iG = rcp64(ac + bc);
            const float Ka = (float)(2.0 * rcp64(ac) * iG);   // without J: applied in FP64
            const float Kb = (float)(2.0 * rcp64(bc) * iG);
            const double r_thr = fmax(tau, kMixedTau) * iG;
            const double fr[3] = {tmid, 0.5 * ac, 0.5 * bc};
            cs32 Bk[3], S[3], Cp[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Bk[c] = sincos32_acc(hx * fr[c]);
                S[c] = sincos32_acc(2.0 * h * fr[c]);
                Cp[c] = sincos32_acc((double)(2 * p0 + 1) * h * fr[c]);
            }
#pragma unroll
            for (int pl = 0; pl < PG; ++pl) {
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const int slot = 2 * pl + sg;
                    cs32 E1, Eu, Ev;
                    if (sg == 1 && p0 + pl == 0) {
                        const double rd = h - hx;   // small radius: direct phases
                        E1 = sincos32_acc(rd * fr[0]);
                        Eu = sincos32_acc(rd * fr[1]);
                        Ev = sincos32_acc(rd * fr[2]);
                    } else {
                        E1 = sg == 0 ? pmul(Cp[0], Bk[0]) : pmulc(Cp[0], Bk[0]);
                        Eu = sg == 0 ? pmul(Cp[1], Bk[1]) : pmulc(Cp[1], Bk[1]);
                        Ev = sg == 0 ? pmul(Cp[2], Bk[2]) : pmulc(Cp[2], Bk[2]);
                    }
                    float Yr, Xr, half = 0.0f;
                    double scale = J;
                    const float r = rr[slot];
                    if ((double)r < r_thr) {
                        // the series in FP64 (its coefficients would carry
                        // the same FP32 rounding for every triangle)
                        const double m = (double)(2 * (p0 + pl) + 1) * h;
                        const double rd = sg == 0 ? m + hx : m - hx;
                        double sre, sim;
                        dd2_series_dev<kMixedSeriesN>(rd * ac, rd * bc, sre, sim);
                        Yr = (float)sre;
                        Xr = (float)sim;
                        // r^2 J stays in FP64: rounded to FP32 it would give
                        // every triangle of equal area the same relative error
                        half = 0.5f;
                        scale = rd * rd * J;
                    } else {
                        const float Pv = Kb * Ev.s;
                        const float Pu = Ka * Eu.s;
                        Yr = __builtin_fmaf(Pv, Ev.s, Pu * Eu.s);
                        Xr = __builtin_fmaf(Pv, Ev.c, -Pu * Eu.c);
                    }
                    const float tre = __builtin_fmaf(half, E1.c, __builtin_fmaf(E1.c, Yr, E1.s * Xr));
                    const float tim = __builtin_fmaf(-half, E1.s, __builtin_fmaf(E1.c, Xr, -E1.s * Yr));
                    acc_re[slot] = __builtin_fma(scale, (double)tre, acc_re[slot]);
                    acc_im[slot] = __builtin_fma(scale, (double)tim, acc_im[slot]);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) Cp[c] = pmul(Cp[c], S[c]);
            }
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) { tot_re[i] += acc_re[i]; tot_im[i] += acc_im[i]; }
    }
}

// General lane, FP64: one node xi = (x, y, z); returns mu^(xi) summed over
// triangles [t_begin, t_end).
HSD_HD void gen_node_f64(const TriRec *A, int64_t nA, const TriRec *B, int64_t t_begin, int64_t t_end,
                         double x, double y, double z, double tau, double &out_re, double &out_im)
{
    double tot_re = 0.0, tot_im = 0.0;
    for (int64_t t0i = t_begin; t0i < t_end; t0i += kTile) {
        double acc_re = 0.0, acc_im = 0.0;
        const int64_t tile_end = (t0i + kTile < t_end) ? t0i + kTile : t_end;
        for (int64_t gi = t0i; gi < tile_end; ++gi) {
            double J;
            const TriRec *rp = tri_at(A, nA, B, gi, J);
            const double t0 = __builtin_fma(x, rp->p0[0], __builtin_fma(y, rp->p0[1], z * rp->p0[2]));
            const double d1 = __builtin_fma(x, rp->e1[0], __builtin_fma(y, rp->e1[1], z * rp->e1[2]));
            const double d2 = __builtin_fma(x, rp->e2[0], __builtin_fma(y, rp->e2[1], z * rp->e2[2]));
            double lo, mid, hi;
            sort3(0.0, d1, d2, lo, mid, hi);
            const double a = mid - lo, b = hi - mid;
            const cs64 E1 = sincos64(t0 + mid);
            double Yr, Xr;
            if (a + b < tau) {
                double fre, fim;
                dd2_series(a, b, fre, fim);
                Yr = J * fre;
                Xr = J * fim;
            } else {
                const double ac = fmax(a, kGapFloor), bc = fmax(b, kGapFloor);
                const double iG = rcp64(ac + bc);
                const double Ka = 2.0 * J * rcp64(ac) * iG;
                const double Kb = 2.0 * J * rcp64(bc) * iG;
                const cs64 Eu = sincos64(0.5 * ac);
                const cs64 Ev = sincos64(0.5 * bc);
                const double Pv = Kb * Ev.s, Pu = Ka * Eu.s;
                Yr = __builtin_fma(Pv, Ev.s, Pu * Eu.s);
                Xr = __builtin_fma(Pv, Ev.c, -Pu * Eu.c);
            }
            acc_re += __builtin_fma(E1.c, Yr, E1.s * Xr);
            acc_im += __builtin_fma(E1.c, Xr, -E1.s * Yr);
        }
        tot_re += acc_re;
        tot_im += acc_im;
    }
    out_re = tot_re;
    out_im = tot_im;
}

// General lane, mixed precision.
HSD_HD void gen_node_mixed(const TriRec *A, int64_t nA, const TriRec *B, int64_t t_begin, int64_t t_end,
                           double x, double y, double z, double tau, double &out_re, double &out_im)
{
    double tot_re = 0.0, tot_im = 0.0;
    for (int64_t t0i = t_begin; t0i < t_end; t0i += kTile) {
        double acc_re = 0.0, acc_im = 0.0;
        const int64_t tile_end = (t0i + kTile < t_end) ? t0i + kTile : t_end;
        for (int64_t gi = t0i; gi < tile_end; ++gi) {
            double J;
            const TriRec *rp = tri_at(A, nA, B, gi, J);
            const double t0 = __builtin_fma(x, rp->p0[0], __builtin_fma(y, rp->p0[1], z * rp->p0[2]));
            const double d1 = __builtin_fma(x, rp->e1[0], __builtin_fma(y, rp->e1[1], z * rp->e1[2]));
            const double d2 = __builtin_fma(x, rp->e2[0], __builtin_fma(y, rp->e2[1], z * rp->e2[2]));
            double lo, mid, hi;
            sort3(0.0, d1, d2, lo, mid, hi);
            const double a = mid - lo, b = hi - mid;
            const cs32 E1 = sincos32_acc(t0 + mid);
            float Yr, Xr, half = 0.0f;
            if (a + b < fmax(tau, kMixedTau)) {
                double sre, sim;
                dd2_series_dev<kMixedSeriesN>(a, b, sre, sim);
                Yr = (float)sre;
                Xr = (float)sim;
                half = 0.5f;
            } else {
                const double ac = fmax(a, kGapFloor32), bc = fmax(b, kGapFloor32);
                const double iG = rcp64(ac + bc);
                const float Ka = (float)(2.0 * rcp64(ac) * iG);
                const float Kb = (float)(2.0 * rcp64(bc) * iG);
                const cs32 Eu = sincos32_acc(0.5 * ac);
                const cs32 Ev = sincos32_acc(0.5 * bc);
                const float Pv = Kb * Ev.s, Pu = Ka * Eu.s;
                Yr = __builtin_fmaf(Pv, Ev.s, Pu * Eu.s);
                Xr = __builtin_fmaf(Pv, Ev.c, -Pu * Eu.c);
            }
            const float tre = __builtin_fmaf(half, E1.c, __builtin_fmaf(E1.c, Yr, E1.s * Xr));
            const float tim = __builtin_fmaf(-half, E1.s, __builtin_fmaf(E1.c, Xr, -E1.s * Yr));
            acc_re = __builtin_fma(J, (double)tre, acc_re);   // J applied in FP64
            acc_im = __builtin_fma(J, (double)tim, acc_im);
        }
        tot_re += acc_re;
        tot_im += acc_im;
    }
    out_re = tot_re;
    out_im = tot_im;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Lane decomposition of the spherical-product kernel: lane = ((g * n_dir) + d)
// * n_half + k, so the 64 lanes of a wave share the panel group g and hold
// 64 / n_half consecutive directions.
template <int PG, int FORM>
__global__ __launch_bounds__(256) void k_direct_sp(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int n_half, int n, int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    constexpr int NS = 2 * PG;
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_lanes = (int64_t)(P / PG) * d_count * n_half;
    const bool active = lane < n_lanes;
    const int64_t L = active ? lane : 0;
    const int k = (int)(L % n_half);
    const int64_t gd = L / n_half;
    const int64_t d = d_begin + gd % d_count;
    const int g = (int)(gd / d_count);
    const int p0 = g * PG;
    const int64_t ntot = nA + nB;
    const int K = gridDim.y;
    const int64_t t_begin = ntot * blockIdx.y / K;
    const int64_t t_end = ntot * (blockIdx.y + 1) / K;
    double tot_re[NS], tot_im[NS];
    if (FORM == HSD_FORM_FP64)
        sp_lane_f64<PG>(A, nA, B, t_begin, t_end, dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2],
                        hx_tab[k], p0, h, tau, tot_re, tot_im);
    else
        sp_lane_mixed<PG>(A, nA, B, t_begin, t_end, dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2],
                          hx_tab[k], p0, h, tau, tot_re, tot_im);
    if (!active) return;
    const double hx = hx_tab[k];
    double2 *out = partial + (int64_t)blockIdx.y * N + (int64_t)d * (P * n);
#pragma unroll
    for (int pl = 0; pl < PG; ++pl) {
        const double m = (double)(2 * (p0 + pl) + 1) * h;
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const int slot = 2 * pl + sg;
            const double r = sg == 0 ? m + hx : m - hx;
            const double inv = 1.0 / (r * r);
            const int j = sg == 0 ? n_half + k : n_half - 1 - k;
            out[(int64_t)(p0 + pl) * n + j] = make_double2(tot_re[slot] * inv, tot_im[slot] * inv);
        }
    }
}

template <int FORM>
__global__ __launch_bounds__(256) void k_direct_gen(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ nodes, int64_t n, int64_t i_begin, int64_t i_count, double tau,
    double2 *__restrict__ partial)
{
    const int64_t i = i_begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < i_begin + i_count;
    const int64_t I = active ? i : 0;
    const int64_t ntot = nA + nB;
    const int K = gridDim.y;
    const int64_t t_begin = ntot * blockIdx.y / K;
    const int64_t t_end = ntot * (blockIdx.y + 1) / K;
    double re, im;
    if (FORM == HSD_FORM_FP64)
        gen_node_f64(A, nA, B, t_begin, t_end, nodes[3 * I], nodes[3 * I + 1], nodes[3 * I + 2], tau, re, im);
    else
        gen_node_mixed(A, nA, B, t_begin, t_end, nodes[3 * I], nodes[3 * I + 1], nodes[3 * I + 2], tau, re, im);
    if (active) partial[(int64_t)blockIdx.y * n + i] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// finalize + reductions
// ---------------------------------------------------------------------------
constexpr int kFinBlock = 256;

__device__ __forceinline__ double wave_sum_fixed(double v)
{
    // butterfly over the 64 lanes in a fixed pattern: every lane ends with the
    // same value, independent of scheduling
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double block_sum_fixed(double v, double *lds)
{
    v = wave_sum_fixed(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) s += lds[i];
    }
    return s;
}

// Per node: mu = sum_k partial[k] (fixed order); R = mu - nu^ (sphere) or mu
// (second mesh already subtracted with sign -1); val = W |R|^2.
// sp: node i = d * n_rad + ir, W = wdir[d] * wtab[ir], nu = nutab[ir];
// general: W = wtab[i], nu = nutab[i].
__global__ __launch_bounds__(kFinBlock) void k_finalize(
    const double2 *__restrict__ partial, int K, int64_t N, int64_t n_rad,
    const double *__restrict__ wdir, const double *__restrict__ wtab,
    const double *__restrict__ nutab, int sphere, double2 *__restrict__ resid,
    double *__restrict__ block_out)
{
    __shared__ double lds[kFinBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (i < N) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < K; ++k) {
            const double2 p = partial[(int64_t)k * N + i];
            re += p.x;
            im += p.y;
        }
        double W, nu;
        if (wdir) {
            const int64_t d = i / n_rad, ir = i - d * n_rad;
            W = wdir[d] * wtab[ir];
            nu = nutab[ir];
        } else {
            W = wtab[i];
            nu = nutab[i];
        }
        if (sphere) re -= nu;
        if (resid) resid[i] = make_double2(re, im);
        val = W * (re * re + im * im);
    }
    const double s = block_sum_fixed(val, lds);
    if (threadIdx.x == 0) block_out[blockIdx.x] = s;
}

// One block: Neumaier sums of a fixed strided subset per thread, then a fixed
// pairwise tree over the threads (values and compensations).
__global__ __launch_bounds__(1024) void k_final_reduce(const double *__restrict__ in, int64_t n,
                                                       double *__restrict__ out)
{
    __shared__ double ls[1024], lc[1024];
    double s = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = in[i];
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    ls[threadIdx.x] = s;
    lc[threadIdx.x] = c;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double a = ls[threadIdx.x], b = ls[threadIdx.x + w];
            const double t = a + b;
            const double e = (fabs(a) >= fabs(b)) ? ((a - t) + b) : ((b - t) + a);
            ls[threadIdx.x] = t;
            lc[threadIdx.x] += lc[threadIdx.x + w] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = ls[0] + lc[0];
}

__global__ void k_sum_partials(const double2 *__restrict__ partial, int K, int64_t N,
                               double2 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < K; ++k) {
        const double2 p = partial[(int64_t)k * N + i];
        re += p.x;
        im += p.y;
    }
    out[i] = make_double2(re, im);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Panels per lane group: FP64 lanes hold 2*PG complex FP64 accumulator pairs,
// so PG = 4 keeps them within 256 VGPRs at 2 waves/SIMD; the mixed form's FP32
// tile sums allow PG = 8 at the same occupancy.
static int pick_pg(int P, int form)
{
    if (form != HSD_FORM_FP64 && P % 8 == 0) return 8;
    if (P % 4 == 0) return 4;
    if (P % 2 == 0) return 2;
    return 1;
}

int choose_k_splits_sp(const hsd_rule *rule, int64_t nt, int form, int num_cu, int req)
{
    if (nt <= 0) return 1;
    if (req > 0) return (int)std::min<int64_t>(req, std::max<int64_t>(1, nt));
    int64_t waves;
    if (wave_kernel_applies(rule)) {
        waves = wave_count(rule);
    } else {
        const int PG = pick_pg(rule->sp.P, form);
        const int64_t lanes = (int64_t)(rule->sp.P / PG) * rule->n_dir * (rule->sp.n / 2);
        waves = (lanes + 63) / 64;
    }
    // aim for >= 8 waves per SIMD (4 SIMDs per CU) and >= 64 triangles per split
    const int64_t target = (int64_t)num_cu * 4 * 8;
    int64_t K = (target + waves - 1) / waves;
    K = std::max<int64_t>(1, std::min<int64_t>(K, (nt + 63) / 64));
    (void)form;
    return (int)std::min<int64_t>(K, 4096);
}

int choose_k_splits_gen(int64_t n, int64_t nt, int num_cu, int req)
{
    if (nt <= 0) return 1;
    if (req > 0) return (int)std::min<int64_t>(req, std::max<int64_t>(1, nt));
    const int64_t waves = (n + 63) / 64;
    const int64_t target = (int64_t)num_cu * 4 * 8;
    int64_t K = (target + waves - 1) / waves;
    K = std::max<int64_t>(1, std::min<int64_t>(K, (nt + 31) / 32));
    return (int)std::min<int64_t>(K, 4096);
}

template <int PG>
static hsd_status launch_sp_pg(hipStream_t st, const MeshPair &mp, const hsd_rule *rule, int form, double tau,
                               int K, int64_t d_begin, int64_t d_count, double2 *partial)
{
    const RuleSP &sp = rule->sp;
    const int n_half = sp.n / 2;
    const int64_t lanes = (int64_t)(sp.P / PG) * d_count * n_half;
    const int64_t blocks = (lanes + 255) / 256;
    if (lanes <= 0) return HSD_OK;
    if (blocks > INT32_MAX || K > 65535) {
        set_error("direct_sp: grid too large (%lld blocks, K=%d)", (long long)blocks, K);
        return HSD_EINVAL;
    }
    dim3 grid((unsigned)blocks, (unsigned)K), block(256);
    if (form == HSD_FORM_FP64)
        hipLaunchKernelGGL((k_direct_sp<PG, HSD_FORM_FP64>), grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           rule->d_dirs.as<const double>(), rule->d_hx.as<const double>(), d_begin, d_count,
                           n_half, sp.n, sp.P, sp.h, tau, rule->n_nodes, partial);
    else
        hipLaunchKernelGGL((k_direct_sp<PG, HSD_FORM_MIXED>), grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           rule->d_dirs.as<const double>(), rule->d_hx.as<const double>(), d_begin, d_count,
                           n_half, sp.n, sp.P, sp.h, tau, rule->n_nodes, partial);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

hsd_status launch_direct_sp_range(hipStream_t st, const MeshPair &mp, const hsd_rule *rule, int form,
                                  double tau, int K, int64_t d_begin, int64_t d_count, double2 *partial)
{
    if (wave_kernel_applies(rule)) return launch_direct_wave(st, mp, rule, form, tau, K, d_begin, d_count, partial);
    switch (pick_pg(rule->sp.P, form)) {
    case 8: return launch_sp_pg<8>(st, mp, rule, form, tau, K, d_begin, d_count, partial);
    case 4: return launch_sp_pg<4>(st, mp, rule, form, tau, K, d_begin, d_count, partial);
    case 2: return launch_sp_pg<2>(st, mp, rule, form, tau, K, d_begin, d_count, partial);
    default: return launch_sp_pg<1>(st, mp, rule, form, tau, K, d_begin, d_count, partial);
    }
}

hsd_status launch_direct_sp(hipStream_t st, const MeshPair &mp, const hsd_rule *rule, int form, double tau,
                            int K, double2 *partial)
{
    return launch_direct_sp_range(st, mp, rule, form, tau, K, 0, rule->n_dir, partial);
}

hsd_status launch_direct_gen_range(hipStream_t st, const MeshPair &mp, const double *nodes, int64_t n,
                                   int form, double tau, int K, int64_t i_begin, int64_t i_count,
                                   double2 *partial)
{
    const int64_t blocks = (i_count + 255) / 256;
    if (i_count <= 0) return HSD_OK;
    if (blocks > INT32_MAX || K > 65535) {
        set_error("direct_gen: grid too large");
        return HSD_EINVAL;
    }
    dim3 grid((unsigned)blocks, (unsigned)K), block(256);
    if (form == HSD_FORM_FP64)
        hipLaunchKernelGGL(k_direct_gen<HSD_FORM_FP64>, grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           nodes, n, i_begin, i_count, tau, partial);
    else
        hipLaunchKernelGGL(k_direct_gen<HSD_FORM_MIXED>, grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           nodes, n, i_begin, i_count, tau, partial);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

hsd_status launch_direct_gen(hipStream_t st, const MeshPair &mp, const double *nodes, int64_t n, int form,
                             double tau, int K, double2 *partial)
{
    return launch_direct_gen_range(st, mp, nodes, n, form, tau, K, 0, n, partial);
}

int64_t finalize_blocks(int64_t n) { return (n + kFinBlock - 1) / kFinBlock; }

hsd_status launch_finalize(hipStream_t st, const hsd_rule *rule, const double *wtab,
                           const double *nutab, const double2 *partial, int K, int64_t n,
                           bool sphere_target, double2 *resid_out, double *block_out,
                           int64_t nblocks)
{
    const bool sp = rule->kind == HSD_RULE_SPHERICAL_PRODUCT;
    if (nblocks > INT32_MAX) {
        set_error("finalize: too many nodes");
        return HSD_EINVAL;
    }
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)nblocks), dim3(kFinBlock), 0, st, partial, K, n,
                       rule->n_rad, sp ? rule->d_wdir.as<const double>() : nullptr, wtab, nutab,
                       sphere_target ? 1 : 0, resid_out, block_out);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

hsd_status launch_final_reduce(hipStream_t st, const double *block_in, int64_t nblocks, double *out)
{
    hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(1024), 0, st, block_in, nblocks, out);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

hsd_status launch_sum_partials(hipStream_t st, const double2 *partial, int K, int64_t n, double2 *out)
{
    if (n <= 0) return HSD_OK;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)blocks), dim3(256), 0, st, partial, K, n, out);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

} // namespace hsd

#ifdef HSD_TEST_HOOKS
// ---------------------------------------------------------------------------
// Host-side self checks: the same lane bodies run on the CPU (not part of the
// public ABI; used by the library's CPU tests, small inputs only).
// ---------------------------------------------------------------------------
namespace hsd {

template <int PG>
static void host_sp_all(const TriRec *A, int64_t nA, const double *dirs, int64_t n_dir, const double *hx_tab,
                        int n, int P, double h, double tau, int form, double *out)
{
    const int n_half = n / 2;
    double tr[2 * PG], ti[2 * PG];
    for (int g = 0; g < P / PG; ++g)
        for (int64_t d = 0; d < n_dir; ++d)
            for (int k = 0; k < n_half; ++k) {
                const int p0 = g * PG;
                if (form == HSD_FORM_FP64)
                    sp_lane_f64<PG>(A, nA, nullptr, 0, nA, dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2],
                                    hx_tab[k], p0, h, tau, tr, ti);
                else
                    sp_lane_mixed<PG>(A, nA, nullptr, 0, nA, dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2],
                                      hx_tab[k], p0, h, tau, tr, ti);
                for (int pl = 0; pl < PG; ++pl)
                    for (int sg = 0; sg < 2; ++sg) {
                        const double m = (double)(2 * (p0 + pl) + 1) * h;
                        const double r = sg == 0 ? m + hx_tab[k] : m - hx_tab[k];
                        const int j = sg == 0 ? n_half + k : n_half - 1 - k;
                        const int64_t q = d * (int64_t)P * n + (int64_t)(p0 + pl) * n + j;
                        out[2 * q] = tr[2 * pl + sg] / (r * r);
                        out[2 * q + 1] = ti[2 * pl + sg] / (r * r);
                    }
            }
}

void build_tri_records(const double *verts, const int32_t *tris, int64_t nt, TriRec *rec);

} // namespace hsd

extern "C" {

// mu^ of a mesh at every node of a spherical product rule given in factored
// form (dirs[n_dir*3], hx_tab[n/2] = h * positive GL nodes), computed on the
// CPU by the kernels' lane bodies.  out[N*2], N = n_dir * P * n.
int hsd__host_transform_sp(const double *verts, const int32_t *tris, int64_t nt, const double *dirs,
                           int64_t n_dir, const double *hx_tab, int n, int P, double h, double tau,
                           int form, double *out)
{
    using namespace hsd;
    std::vector<TriRec> rec((size_t)nt);
    build_tri_records(verts, tris, nt, rec.data());
    switch (pick_pg(P, form)) {
    case 8: host_sp_all<8>(rec.data(), nt, dirs, n_dir, hx_tab, n, P, h, tau, form, out); break;
    case 4: host_sp_all<4>(rec.data(), nt, dirs, n_dir, hx_tab, n, P, h, tau, form, out); break;
    case 2: host_sp_all<2>(rec.data(), nt, dirs, n_dir, hx_tab, n, P, h, tau, form, out); break;
    default: host_sp_all<1>(rec.data(), nt, dirs, n_dir, hx_tab, n, P, h, tau, form, out); break;
    }
    return 0;
}

// mu^ of a mesh at arbitrary nodes, CPU run of the general lane body.
int hsd__host_transform_gen(const double *verts, const int32_t *tris, int64_t nt, const double *nodes,
                            int64_t n, double tau, int form, double *out)
{
    using namespace hsd;
    std::vector<TriRec> rec((size_t)nt);
    build_tri_records(verts, tris, nt, rec.data());
    for (int64_t i = 0; i < n; ++i) {
        if (form == HSD_FORM_FP64)
            gen_node_f64(rec.data(), nt, nullptr, 0, nt, nodes[3 * i], nodes[3 * i + 1], nodes[3 * i + 2], tau,
                         out[2 * i], out[2 * i + 1]);
        else
            gen_node_mixed(rec.data(), nt, nullptr, 0, nt, nodes[3 * i], nodes[3 * i + 1], nodes[3 * i + 2], tau,
                           out[2 * i], out[2 * i + 1]);
    }
    return 0;
}

void hsd__host_sincos64(const double *x, int64_t n, double *c, double *s)
{
    for (int64_t i = 0; i < n; ++i) {
        const hsd::cs64 r = hsd::sincos64(x[i]);
        c[i] = r.c;
        s[i] = r.s;
    }
}

void hsd__host_sincos64_tab(const double *x, int64_t n, double *c, double *s)
{
    hsd::cs64 turn[32];
    for (int k = 0; k < 32; ++k) turn[k] = hsd::turn16(k);
    for (int64_t i = 0; i < n; ++i) {
        const hsd::cs64 r = hsd::sincos64_tab(x[i], turn);
        c[i] = r.c;
        s[i] = r.s;
    }
}

void hsd__host_sincos32(const double *x, int64_t n, float *c, float *s)
{
    for (int64_t i = 0; i < n; ++i) {
        const hsd::cs32 r = hsd::sincos32_acc(x[i]);
        c[i] = r.c;
        s[i] = r.s;
    }
}

} // extern "C"
#endif // HSD_TEST_HOOKS
