// hsd_direct_wave.hip -- direct-sum kernel with one wavefront per direction
// for spherical-product rules with 16 Gauss-Legendre nodes per panel.
//
// Same arithmetic as the lane bodies of hsd_direct.hip (exact triangle
// transform as J * e[z0,z1,z2], sorted phases, closed branch above tau,
// series below, r^2-scaled accumulation), organised so the per-(triangle,
// direction) work is shared by the whole wave instead of recomputed by
// every lane:
//
//   * a wave owns one direction n and 8*PG consecutive panels; lane
//     (k, g) = (lane % 8, lane / 8) owns the node pair m_p +- h x_k of its
//     PG panels p = w0 + g*PG + pl (2*PG nodes);
//   * triangles are processed in batches of 8.  Producer step: lane
//     (t, j) = (lane / 8, lane % 8) computes, for triangle t of the batch,
//     exp(-i h x_j c) and the panel-centre phases exp(-i m_p c) of its PG
//     panels (panels w0 + j*PG + q in the FP64 form, w0 + j + 8 q in the
//     mixed form), for the three constants c = theta_mid, a/2, b/2 of the
//     triangle and direction, and stores them with the triangle's scale
//     factors in LDS;
//   * consumer step: every lane forms its node phases by one complex product
//     per constant and node and accumulates, reading the batch from LDS.
//
// Per-lane sums use FP64 tiles of 32 triangles merged into running totals
// (the mixed form adds its FP32 contributions in FP64 too); K triangle
// splits on grid.y as in hsd_direct.hip.
#include <type_traits>
#include <vector>

#include "hsd_internal.hpp"
#include "hsd_math.hpp"

namespace hsd {

namespace wv {

constexpr int kTB = 8;        // triangles per batch
constexpr int kNH = 8;        // node pairs per panel (16 GL nodes)
constexpr int kTileBatches = 4;   // batches per FP64 tile sum (32 triangles)
constexpr double kGapFloor = 1e-150;
constexpr double kGapFloor32 = 1e-18;

// Per-(triangle, direction) constants in LDS.  ce/co are the coefficients of
// the divided-difference power series as a polynomial in the radius r:
// Re = sum_m ce[m] r^(2m), Im = r sum_m co[m] r^(2m) (see series_coefs).
// FP64 form: series through r^7; the first omitted term is below
// 9 G^8 / 10! of the leading 1/2, 1e-16 at the largest threshold the form
// accepts (G < 0.05) and 2.5e-22 at the default 0.01.  For thresholds up to
// kTauNC3 the consumer sums only through r^5 (first omitted term below
// 7 G^6 / 8! of the leading 1/2: 4e-15 at 0.015, 3.5e-16 at 0.01).
constexpr int kNC64 = 4;
constexpr double kTauNC3 = 0.015;
constexpr int kNC32 = (kMixedSeriesN + 1) / 2;  // through r^kMixedSeriesN (mixed form)
struct Scal64 { double rthr, pad; double ce[kNC64], co[kNC64]; };   // ce, co carry the factor |J|
struct Scal32 { float rthr, Ka, Kb, c0lo; float ce[kNC32], co[kNC32]; };   // Ka, Kb, ce, co carry |J|

template <int PG> struct Batch64 {
    Scal64 sc[kTB];
    cs64 Bk[kTB][kNH][3];
    cs64 Cp[kTB][kNH * PG][3];
};
template <int PG> struct Batch32 {
    Scal32 sc[kTB];
    cs32 Bk[kTB][kNH][3];
    cs32 Cp[kTB][kNH * PG][3];
};

// Per-(triangle, direction) constants: sorted gaps (floored), theta_mid and
// the closed-branch scale factors.
struct TriDir {
    double tmid, ac, bc, iG, J;
};

HSD_HD TriDir tri_dir(const TriRec &T, double J, double nx, double ny, double nz, double floor)
{
    const double t0 = __builtin_fma(nx, T.p0[0], __builtin_fma(ny, T.p0[1], nz * T.p0[2]));
    const double d1 = __builtin_fma(nx, T.e1[0], __builtin_fma(ny, T.e1[1], nz * T.e1[2]));
    const double d2 = __builtin_fma(nx, T.e2[0], __builtin_fma(ny, T.e2[1], nz * T.e2[2]));
    double lo, mid, hi;
    sort3(0.0, d1, d2, lo, mid, hi);
    TriDir r;
    r.ac = fmax(mid - lo, floor);
    r.bc = fmax(hi - mid, floor);
    r.tmid = t0 + mid;
    r.iG = rcp64(r.ac + r.bc);
    r.J = J;
    return r;
}

// Coefficients of the second divided difference of exp at (i a, 0, -i b) as
// a power series in r for a = r ac, b = r bc:  sum_n (-i)^n r^n h_n with
// h_n = H_n(ac, bc) / (n+2)!, H_n = sum_{m<=n} (-ac)^m bc^(n-m) (complete
// homogeneous polynomial, by the recurrence H_n = bc H_{n-1} + (-ac)^n).
// Split by parity: ce[m] = (-1)^m h_{2m}, co[m] = (-1)^(m+1) h_{2m+1}, m < NC.
// Through n = 2 NC - 1: the first omitted term is below
// (2 NC + 1) G^(2 NC) / (2 NC + 2)! relative to the leading 1/2, with
// G = r (ac + bc) the scaled phase spread.
// The scale factor rides along in H and the powers (H_0 = scale).
template <int NC>
HSD_HD void series_coefs(double ac, double bc, double scale, double ce[NC], double co[NC])
{
    double H = scale, pw = scale;
    ce[0] = 0.5 * scale;
#pragma unroll
    for (int n = 1; n <= 2 * NC - 1; ++n) {
        pw *= -ac;
        H = __builtin_fma(H, bc, pw);
        const double hn = H * inv_factorial(n + 2);
        if (n & 1) co[n >> 1] = ((n >> 1) & 1) ? hn : -hn;
        else ce[n >> 1] = ((n >> 1) & 1) ? -hn : hn;
    }
}

// Even/odd polynomial of the series at r (r2 = r^2) through its first NC
// coefficients of each parity: returns Re, Im / r.
template <int NC, typename T>
HSD_HD void series_eval(const T ce[kNC64], const T co[kNC64], T r2, T &pe, T &po)
{
    pe = ce[NC - 1];
    po = co[NC - 1];
#pragma unroll
    for (int m = NC - 2; m >= 0; --m) {
        pe = pe * r2 + ce[m];
        po = po * r2 + co[m];
    }
}

// Phase e^{-i h c} of the first panel's centre, held by the first lane of
// each group of 8 producer lanes (one triangle) when the wave starts at
// panel 0: broadcast within the group by an LDS swizzle (bit-mask mode, and
// mask 0x18: every lane reads lane (lane & ~7) of its half-wave).  The host
// emulation recomputes what that lane computed.
HSD_HD cs64 group_first_phase(cs64 own, double hc, const cs64 *turn)
{
#if defined(__HIP_DEVICE_COMPILE__)
    (void)hc;
    (void)turn;
    cs64 r;
    r.c = __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(own.c), 0x18),
                           __builtin_amdgcn_ds_swizzle(__double2loint(own.c), 0x18));
    r.s = __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(own.s), 0x18),
                           __builtin_amdgcn_ds_swizzle(__double2loint(own.s), 0x18));
    return r;
#else
    (void)own;
    return sincos64_tab(hc, turn);
#endif
}

// Producer, FP64: part j of a triangle's batch entry (the half-node phases
// of node j and the centre phases of panels w0 + j PG .. w0 + j PG + PG-1).
// ONE: the wave covers all panels of its direction (w0 = 0); the second
// panel's phase is then the first one's times e^{-2 i h c}, the square of the
// group's panel-0 phase, instead of another sin/cos.
//
// The closed branch needs K_a sin^2(r a/2), K_a sin(r a/2) cos(r a/2) and
// the same for b, with K_a = 2 |J| / (G a), K_b = 2 |J| / (G b).  The
// centre phases of the two half gaps are stored times sqrt(K_a), sqrt(K_b),
// so the consumer's phase products give sqrt(K) e^{-i r g/2} and the four
// terms are two squares and two products of their parts.  The sign of J
// (-1 for a second mesh) rides on the theta_mid half-node phase, the series
// coefficients carry |J|.
template <int PG, bool ONE>
HSD_HD void produce64(const TriDir &td, double h, const double *hx_tab, int j, int w0, double tau,
                      const cs64 *turn, Scal64 *sc, cs64 Bk[3], cs64 Cp[PG][3])
{
    const double fr[3] = {td.tmid, 0.5 * td.ac, 0.5 * td.bc};
    const double hx = hx_tab[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Bk[c] = sincos64_tab(hx * fr[c], turn);
        Cp[0][c] = sincos64_tab((double)(2 * (w0 + j * PG) + 1) * h * fr[c], turn);
        if constexpr (ONE && PG > 1) {
            const cs64 e1 = group_first_phase(Cp[0][c], h * fr[c], turn);
            const cs64 step = pmul(e1, e1);
#pragma unroll
            for (int q = 1; q < PG; ++q) Cp[q][c] = pmul(Cp[q - 1][c], step);
        } else {
#pragma unroll
            for (int q = 1; q < PG; ++q)
                Cp[q][c] = sincos64_tab((double)(2 * (w0 + j * PG + q) + 1) * h * fr[c], turn);
        }
    }
    // 1/ac and 1/bc from one reciprocal of ac bc (both gaps are floored at
    // 1e-150, so the product stays a normal number)
    const double aJ = fabs(td.J);
    const double rab = rcp64(td.ac * td.bc);
    const double t = 2.0 * aJ * td.iG;
    const double ska = sqrt_pos64(t * (td.bc * rab)), skb = sqrt_pos64(t * (td.ac * rab));
    if (td.J < 0.0) Bk[0] = cs64{-Bk[0].c, -Bk[0].s};
#pragma unroll
    for (int q = 0; q < PG; ++q) {
        Cp[q][1] = cs64{ska * Cp[q][1].c, ska * Cp[q][1].s};
        Cp[q][2] = cs64{skb * Cp[q][2].c, skb * Cp[q][2].s};
    }
    if (sc) {
        sc->rthr = tau * td.iG;
        sc->pad = 0.0;
        series_coefs<kNC64>(td.ac, td.bc, aJ, sc->ce, sc->co);
    }
}

// Consumer, FP64: one triangle into the lane's 2*PG slots (slot 2*pl + sg).
// Every node's phases are products of a panel-centre and a half-node phase,
// also for the small-radius node h - h x_k of panel 0: the product carries an
// absolute error of a few ulp in its sine, which the closed branch (taken
// only for r G >= tau) turns into a relative error below ~eps / tau, the
// same class as the branch's own cancellation; below tau only the
// theta_mid phase enters.
//
// The series branch replaces the closed one where r < tau / G.  Within a
// lane the slot (pl 0, minus) has the smallest radius; r_others is the
// smallest radius of any other slot over the whole wave ((2 w0 + 1) h +
// h x_0), so when the triangle's threshold is not above it only that slot
// can take the series, and the others skip their compare.  nc3: thresholds
// up to kTauNC3, series through r^5.
template <int PG>
HSD_HD void consume64(const Scal64 &sc, const cs64 Bk[3], const cs64 (*Cp)[3], double h,
                      double hx, int pbase, double r_others, bool nc3, double *acc_re, double *acc_im)
{
    constexpr int NS = 2 * PG;
    double Yr[NS], Xr[NS], rs[NS];
#pragma unroll
    for (int pl = 0; pl < PG; ++pl) {
        const double m = (double)(2 * (pbase + pl) + 1) * h;
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const int slot = 2 * pl + sg;
            rs[slot] = sg == 0 ? m + hx : m - hx;
            // E[1], E[2] carry sqrt(K_a), sqrt(K_b) (see produce64)
            const cs64 E1 = sg == 0 ? pmul(Cp[pl][1], Bk[1]) : pmulc(Cp[pl][1], Bk[1]);
            const cs64 E2 = sg == 0 ? pmul(Cp[pl][2], Bk[2]) : pmulc(Cp[pl][2], Bk[2]);
            Yr[slot] = __builtin_fma(E2.s, E2.s, E1.s * E1.s);
            Xr[slot] = __builtin_fma(E2.s, E2.c, -(E1.s * E1.c));
        }
    }
    auto series = [&](int slot) {
        const double r = rs[slot], r2 = r * r;
        double pe, po;
        if (nc3)
            series_eval<3>(sc.ce, sc.co, r2, pe, po);
        else
            series_eval<kNC64>(sc.ce, sc.co, r2, pe, po);
        Yr[slot] = r2 * pe;
        Xr[slot] = r2 * r * po;
    };
    if (rs[1] < sc.rthr) series(1);
    if (sc.rthr > r_others) {
#pragma unroll
        for (int slot = 0; slot < NS; ++slot)
            if (slot != 1 && rs[slot] < sc.rthr) series(slot);
    }
#pragma unroll
    for (int pl = 0; pl < PG; ++pl) {
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const int slot = 2 * pl + sg;
            const cs64 E0 = sg == 0 ? pmul(Cp[pl][0], Bk[0]) : pmulc(Cp[pl][0], Bk[0]);
            acc_re[slot] = __builtin_fma(E0.c, Yr[slot], __builtin_fma(E0.s, Xr[slot], acc_re[slot]));
            acc_im[slot] = __builtin_fma(E0.c, Xr[slot], __builtin_fma(-E0.s, Yr[slot], acc_im[slot]));
        }
    }
}

// Producer, mixed: FP32 phases from FP64-reduced angles.  Cp is the
// triangle's whole row, indexed by panel offset in the wave; part j fills
// panels j + kNH q.  The sign of J (-1 for a second mesh) rides on the
// theta_mid phase row; the closed-branch factors K_a = 2 |J| / (G a),
// K_b = 2 |J| / (G b) and the series coefficients carry |J|, each rounded
// once to FP32 (a relative error that differs between directions, since the
// gaps do).  The series' constant term |J|/2 does not depend on the
// direction, so its FP32 rounding would be the same for every triangle of
// equal area (a symmetric mesh has few distinct areas) and would not
// average out: it is kept as the two-float pair ce[0] + c0lo.
template <int PG>
HSD_HD void produce32(const TriDir &td, double h, const double *hx_tab, int j, int w0, double tau,
                      Scal32 *sc, cs32 Bk[3], cs32 (*Cp)[3])
{
    const double fr[3] = {td.tmid, 0.5 * td.ac, 0.5 * td.bc};
    const double hx = hx_tab[j];
    const float sgn = td.J < 0.0 ? -1.0f : 1.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Bk[c] = sincos32_acc(hx * fr[c]);
#pragma unroll
        for (int q = 0; q < PG; ++q) {
            cs32 e = sincos32_acc((double)(2 * (w0 + j + kNH * q) + 1) * h * fr[c]);
            if (c == 0) e = cs32{sgn * e.c, sgn * e.s};
            Cp[j + kNH * q][c] = e;
        }
    }
    if (sc) {
        const double aJ = fabs(td.J);
        const double rab = rcp64(td.ac * td.bc);   // gaps floored at 1e-18
        const double t = 2.0 * aJ * td.iG;
        sc->Ka = (float)(t * (td.bc * rab));
        sc->Kb = (float)(t * (td.ac * rab));
        sc->rthr = (float)(fmax(tau, kMixedTau) * td.iG);   // decides the branch only
        double ce[kNC32], co[kNC32];
        series_coefs<kNC32>(td.ac, td.bc, aJ, ce, co);
        sc->ce[0] = (float)ce[0];
        sc->c0lo = (float)(ce[0] - (double)sc->ce[0]);
#pragma unroll
        for (int m = 1; m < kNC32; ++m) sc->ce[m] = (float)ce[m];
#pragma unroll
        for (int m = 0; m < kNC32; ++m) sc->co[m] = (float)co[m];
    }
}

// Consumer, mixed: FP32 node arithmetic.  The closed branch's terms come out
// scaled by J and r^2 and are summed in FP32 over one batch of 8 triangles
// (acc), which the caller flushes into the FP64 running totals (tot).  The
// series branch's J-scaled terms are added to tot directly, times r^2 in
// FP64: at small r G all triangles' terms are close to J/2 with nearly the
// same phase, so an FP32 partial sum over a batch would grow linearly and
// its rounding would outweigh the terms' own; and r^2 rounded to FP32 would
// give every contribution of a node the same relative error.
//
// Lane layout (mixed form): lane = (po, sg, k) = (lane / 16, lane / 8 % 2,
// lane % 8) holds node m_p + h x_k (sg = 0) or m_p - h x_k (sg = 1) of the
// panels p = w0 + po + 4 q, slot q < 2 PG.  A slot of the wave then covers a
// quarter of the wave's radial range, so that the series threshold r G = tau
// splits one slot per triangle and the others take one branch only.  The
// half-gap phases are formed only where some lane takes the closed branch.
//
// All node phases are products of a panel-centre and a node-offset phase,
// also for the small-radius nodes h - h x_k of panel 0, whose small half-gap
// sines then carry an absolute FP32 rounding: the closed branch (r G >= 0.75
// in this form) enlarges it by at most 1 / (r G), the size of the rounding
// every other node's closed branch carries.
template <int PG>
HSD_HD void consume32(const Scal32 &scr, const cs32 Bk[3], const cs32 (*Cp)[3],
                      const float *rf, const float *r2f, const double *r2d, bool conj, float *acc_re,
                      float *acc_im, double *tot_re, double *tot_im)
{
    constexpr int NS = 2 * PG;
    const Scal32 sc = scr;   // one read of the triangle's constants per triangle
    cs32 B[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) B[c] = cs32{Bk[c].c, conj ? -Bk[c].s : Bk[c].s};
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const cs32 E0 = pmul(Cp[4 * q][0], B[0]);
        if (rf[q] < sc.rthr) {
            // Re of the series minus its constant term; the constant term
            // (J/2) is added last, in one fused step with the rest of the
            // product already summed, so that the rounding sees the exact
            // total (J/2 rounded first and a sub-ulp rest added after it
            // would err the same way for every triangle of a node)
            const float r2 = r2f[q];
            float pe = sc.ce[kNC32 - 1], po = sc.co[kNC32 - 1];
#pragma unroll
            for (int m = kNC32 - 2; m >= 1; --m) pe = __builtin_fmaf(pe, r2, sc.ce[m]);
#pragma unroll
            for (int m = kNC32 - 2; m >= 0; --m) po = __builtin_fmaf(po, r2, sc.co[m]);
            const float Yr = pe * r2;
            const float Xr = rf[q] * po;
            const float yr = Yr + sc.c0lo;
            const float tre = __builtin_fmaf(sc.ce[0], E0.c, __builtin_fmaf(E0.c, yr, E0.s * Xr));
            const float tim = __builtin_fmaf(-sc.ce[0], E0.s, __builtin_fmaf(E0.c, Xr, -E0.s * yr));
            tot_re[q] = __builtin_fma(r2d[q], (double)tre, tot_re[q]);
            tot_im[q] = __builtin_fma(r2d[q], (double)tim, tot_im[q]);
        } else {
            const cs32 E1 = pmul(Cp[4 * q][1], B[1]);
            const cs32 E2 = pmul(Cp[4 * q][2], B[2]);
            const float Pv = sc.Kb * E2.s;
            const float Pu = sc.Ka * E1.s;
            const float Yr = __builtin_fmaf(Pv, E2.s, Pu * E1.s);
            const float Xr = __builtin_fmaf(Pv, E2.c, -Pu * E1.c);
            acc_re[q] = __builtin_fmaf(E0.c, Yr, __builtin_fmaf(E0.s, Xr, acc_re[q]));
            acc_im[q] = __builtin_fmaf(E0.c, Xr, __builtin_fmaf(-E0.s, Yr, acc_im[q]));
        }
    }
}

// Radii of a mixed-form lane's slots (panels w0 + po + 4 q, sign sg) in
// FP32, and their squares in FP32 and FP64.
template <int PG>
HSD_HD void mixed_lane_radii(int w0, int po, int sg, double h, double hx, float *rf, float *r2f, double *r2d)
{
#pragma unroll
    for (int q = 0; q < 2 * PG; ++q) {
        const double m = (double)(2 * (w0 + po + 4 * q) + 1) * h;
        const double rd = sg == 0 ? m + hx : m - hx;
        rf[q] = (float)rd;
        r2d[q] = rd * rd;
        r2f[q] = (float)r2d[q];
    }
}

// Each wave produces and consumes its own LDS batch, so the two steps only
// need ordering among the lanes of that wave: a wavefront-scope fence (the
// compiler waits for the wave's LDS writes before its later reads).  Waves of
// a block never wait for each other.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

HSD_HD const TriRec *tri_at(const TriRec *A, int64_t nA, const TriRec *B, int64_t gi, double &J)
{
    const bool inA = gi < nA;
    const TriRec *rp = inA ? (A + gi) : (B + (gi - nA));
    J = inA ? rp->J : -rp->J;
    return rp;
}

} // namespace wv

// ---------------------------------------------------------------------------
// kernel body: 4 waves per block, one direction (and panel window) per wave
// ---------------------------------------------------------------------------
template <int PG, int FORM, bool ONE>
__device__ __forceinline__ void direct_wave_body(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    using namespace wv;
    constexpr int NS = 2 * PG;
    constexpr bool F64 = FORM == HSD_FORM_FP64;
    __shared__ typename std::conditional<F64, Batch64<PG>, Batch32<PG>>::type lds[4];
    __shared__ cs64 turn[F64 ? 32 : 1];     // e^{i k pi/16} for the FP64 sin/cos
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if constexpr (F64) {
        if (threadIdx.x < 32) turn[threadIdx.x] = turn16((int)threadIdx.x);
        __syncthreads();
    }
    const int wpd = P / (kNH * PG);                 // waves per direction
    const int64_t gw = (int64_t)blockIdx.x * 4 + w;
    const bool valid = gw < d_count * wpd;
    const int64_t GW = valid ? gw : 0;
    const int64_t d = d_begin + GW / wpd;
    const int w0 = (int)(GW % wpd) * kNH * PG;       // first panel of the wave
    const double nx = dirs[3 * d], ny = dirs[3 * d + 1], nz = dirs[3 * d + 2];
    const int k = lane & 7, g = lane >> 3;             // consumer roles
    const int pt = lane >> 3, pj = lane & 7;           // producer roles
    const double hx = hx_tab[k];
    // FP64 consumer slots (pl, sg) hold panel pbase + pl; mixed-form lanes
    // are laid out as (po, sg, k), see consume32
    const int pbase = w0 + g * PG;
    const int po = lane >> 4, sgl = (lane >> 3) & 1;
    float rf[F64 ? 1 : NS], r2f[F64 ? 1 : NS];
    double r2d[F64 ? 1 : NS];
    const double r_others = (double)(2 * w0 + 1) * h + hx_tab[0];   // see consume64
    const bool nc3 = tau <= kTauNC3;
    if constexpr (!F64) mixed_lane_radii<PG>(w0, po, sgl, h, hx, rf, r2f, r2d);
    auto &L = lds[w];

    const int64_t ntot = nA + nB;
    const int K = gridDim.y;
    const int64_t t_begin = ntot * blockIdx.y / K;
    const int64_t t_end = ntot * (blockIdx.y + 1) / K;

    // FP64 form: FP64 tile sums over kTileBatches batches merged into the
    // running totals; mixed form: the closed branch's FP32 sums over one
    // batch flushed into the FP64 running totals after every batch (the
    // series branch adds to the running totals directly, see consume32)
    using Acc = typename std::conditional<F64, double, float>::type;
    double tot_re[NS], tot_im[NS];
    Acc acc_re[NS], acc_im[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) { tot_re[i] = 0.0; tot_im[i] = 0.0; acc_re[i] = 0; acc_im[i] = 0; }

    int nb = 0;
    for (int64_t tb = t_begin; tb < t_end; tb += kTB) {
        const int nvalid = (int)((t_end - tb) < kTB ? (t_end - tb) : kTB);
        {   // produce
            const int64_t gi = tb + (pt < nvalid ? pt : 0);
            double J;
            const TriRec *rp = wv::tri_at(A, nA, B, gi, J);
            const TriDir td = tri_dir(*rp, J, nx, ny, nz, F64 ? kGapFloor : kGapFloor32);
            if constexpr (F64)
                produce64<PG, ONE>(td, h, hx_tab, pj, w0, tau, turn, pj == 0 ? &L.sc[pt] : nullptr, L.Bk[pt][pj],
                                   &L.Cp[pt][pj * PG]);
            else
                produce32<PG>(td, h, hx_tab, pj, w0, tau, pj == 0 ? &L.sc[pt] : nullptr, L.Bk[pt][pj],
                              L.Cp[pt]);
        }
        wave_lds_sync();
        for (int t = 0; t < nvalid; ++t) {
            if constexpr (F64)
                consume64<PG>(L.sc[t], L.Bk[t][k], &L.Cp[t][g * PG], h, hx, pbase, r_others, nc3, acc_re, acc_im);
            else
                consume32<PG>(L.sc[t], L.Bk[t][k], &L.Cp[t][po], rf, r2f, r2d, sgl == 1, acc_re, acc_im, tot_re,
                              tot_im);
        }
        wave_lds_sync();
        if constexpr (F64) {
            if (++nb == kTileBatches) {
                nb = 0;
#pragma unroll
                for (int i = 0; i < NS; ++i) {
                    tot_re[i] += acc_re[i];
                    tot_im[i] += acc_im[i];
                    acc_re[i] = 0.0;
                    acc_im[i] = 0.0;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                tot_re[i] += (double)acc_re[i];
                tot_im[i] += (double)acc_im[i];
                acc_re[i] = 0.0f;
                acc_im[i] = 0.0f;
            }
        }
    }
    if constexpr (F64) {
#pragma unroll
        for (int i = 0; i < NS; ++i) { tot_re[i] += acc_re[i]; tot_im[i] += acc_im[i]; }
    }
    if (!valid) return;
    double2 *out = partial + (int64_t)blockIdx.y * N + d * (int64_t)(P * 2 * kNH);
#pragma unroll
    for (int slot = 0; slot < NS; ++slot) {
        // slot -> (panel, sign): (pbase + slot / 2, slot % 2) in FP64,
        // (w0 + po + 4 slot, sgl) in the mixed form
        const int p = F64 ? pbase + slot / 2 : w0 + po + 4 * slot;
        const int sg = F64 ? slot % 2 : sgl;
        const double m = (double)(2 * p + 1) * h;
        const double r = sg == 0 ? m + hx : m - hx;
        const double inv = 1.0 / (r * r);
        const int jn = sg == 0 ? kNH + k : kNH - 1 - k;
        out[(int64_t)p * (2 * kNH) + jn] = make_double2(tot_re[slot] * inv, tot_im[slot] * inv);
    }
}

// FP64 form: its LDS batch (9.75 KB per wave, 39.5 KB per block) allows 4
// blocks per CU.  ONE: one wave per direction (the wave starts at panel 0).
template <int PG, bool ONE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_direct_wave(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    direct_wave_body<PG, HSD_FORM_FP64, ONE>(A, nA, B, nB, dirs, hx_tab, d_begin, d_count, P, h, tau, N, partial);
}

// Mixed form: its 7 KB of LDS per wave leave the registers as the limit;
// held to 128 VGPRs (4 waves per SIMD; a few spills in the producer) it runs
// about 7% faster than at the 141 it would take.
template <int PG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_direct_wave_mixed(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    direct_wave_body<PG, HSD_FORM_MIXED, false>(A, nA, B, nB, dirs, hx_tab, d_begin, d_count, P, h, tau, N, partial);
}

bool wave_kernel_applies(const hsd_rule *rule)
{
    return rule->kind == HSD_RULE_SPHERICAL_PRODUCT && rule->sp.n == 16 && rule->sp.P % wv::kNH == 0;
}

static int wave_pg(const hsd_rule *rule) { return rule->sp.P % (2 * wv::kNH) == 0 ? 2 : 1; }

int64_t wave_count(const hsd_rule *rule)
{
    const int PG = wave_pg(rule);
    return rule->n_dir * (rule->sp.P / (wv::kNH * PG));
}

template <int PG>
static hsd_status launch_wave_pg(hipStream_t st, const MeshPair &mp, const hsd_rule *rule, int form, double tau,
                                 int K, int64_t d_begin, int64_t d_count, double2 *partial)
{
    const int wpd = rule->sp.P / (wv::kNH * PG);
    const int64_t waves = d_count * wpd;
    const int64_t blocks = (waves + 3) / 4;
    if (waves <= 0) return HSD_OK;
    if (blocks > INT32_MAX || K > 65535) {
        set_error("direct_wave: grid too large");
        return HSD_EINVAL;
    }
    dim3 grid((unsigned)blocks, (unsigned)K), block(256);
    // the single-wave variant differs only where a lane holds two panels
    constexpr bool kOne = PG > 1;
    if (form == HSD_FORM_FP64 && kOne && wpd == 1)
        hipLaunchKernelGGL((k_direct_wave<PG, kOne>), grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           rule->d_dirs.as<const double>(), rule->d_hx.as<const double>(), d_begin, d_count,
                           rule->sp.P, rule->sp.h, tau, rule->n_nodes, partial);
    else if (form == HSD_FORM_FP64)
        hipLaunchKernelGGL((k_direct_wave<PG, false>), grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           rule->d_dirs.as<const double>(), rule->d_hx.as<const double>(), d_begin, d_count,
                           rule->sp.P, rule->sp.h, tau, rule->n_nodes, partial);
    else
        hipLaunchKernelGGL((k_direct_wave_mixed<PG>), grid, block, 0, st, mp.A, mp.nA, mp.B, mp.nB,
                           rule->d_dirs.as<const double>(), rule->d_hx.as<const double>(), d_begin, d_count,
                           rule->sp.P, rule->sp.h, tau, rule->n_nodes, partial);
    HSD_HIP_TRY(hipGetLastError());
    return HSD_OK;
}

hsd_status launch_direct_wave(hipStream_t st, const MeshPair &mp, const hsd_rule *rule, int form, double tau,
                              int K, int64_t d_begin, int64_t d_count, double2 *partial)
{
    return wave_pg(rule) == 2 ? launch_wave_pg<2>(st, mp, rule, form, tau, K, d_begin, d_count, partial)
                              : launch_wave_pg<1>(st, mp, rule, form, tau, K, d_begin, d_count, partial);
}

#ifdef HSD_TEST_HOOKS
// ---------------------------------------------------------------------------
// host emulation of one direction (self checks)
// ---------------------------------------------------------------------------
template <int PG, bool F64>
static void host_wave_dir(const TriRec *A, int64_t nA, double nx, double ny, double nz, const double *hx_tab,
                          int P, double h, double tau, double *out /* [P*16*2] */)
{
    using namespace wv;
    constexpr int NS = 2 * PG;
    const int wpd = P / (kNH * PG);
    std::vector<Batch64<PG>> b64(1);
    std::vector<Batch32<PG>> b32(1);
    cs64 turn[32];
    for (int k = 0; k < 32; ++k) turn[k] = turn16(k);
    for (int wi = 0; wi < wpd; ++wi) {
        const int w0 = wi * kNH * PG;
        std::vector<double> tre(64 * NS, 0.0), tim(64 * NS, 0.0);
        std::vector<double> are(64 * NS, 0.0), aim(64 * NS, 0.0);
        std::vector<float> fre(64 * NS, 0.0f), fim(64 * NS, 0.0f);
        int nb = 0;
        for (int64_t tb = 0; tb < nA; tb += kTB) {
            const int nvalid = (int)std::min<int64_t>(kTB, nA - tb);
            for (int lane = 0; lane < 64; ++lane) {
                const int pt = lane >> 3, pj = lane & 7;
                double J;
                const TriRec *rp = wv::tri_at(A, nA, nullptr, tb + (pt < nvalid ? pt : 0), J);
                const TriDir td = tri_dir(*rp, J, nx, ny, nz, F64 ? kGapFloor : kGapFloor32);
                if (F64) {
                    auto &L = b64[0];
                    if (wpd == 1)
                        produce64<PG, true>(td, h, hx_tab, pj, w0, tau, turn, pj == 0 ? &L.sc[pt] : nullptr,
                                            L.Bk[pt][pj], &L.Cp[pt][pj * PG]);
                    else
                        produce64<PG, false>(td, h, hx_tab, pj, w0, tau, turn, pj == 0 ? &L.sc[pt] : nullptr,
                                             L.Bk[pt][pj], &L.Cp[pt][pj * PG]);
                } else {
                    auto &L = b32[0];
                    produce32<PG>(td, h, hx_tab, pj, w0, tau, pj == 0 ? &L.sc[pt] : nullptr, L.Bk[pt][pj],
                                  L.Cp[pt]);
                }
            }
            for (int lane = 0; lane < 64; ++lane) {
                const int k = lane & 7, g = lane >> 3;
                const int pbase = w0 + g * PG;
                const int po = lane >> 4, sgl = (lane >> 3) & 1;
                float rf[NS], r2f[NS];
                double r2d[NS];
                mixed_lane_radii<PG>(w0, po, sgl, h, hx_tab[k], rf, r2f, r2d);
                for (int t = 0; t < nvalid; ++t) {
                    if (F64) {
                        auto &L = b64[0];
                        consume64<PG>(L.sc[t], L.Bk[t][k], &L.Cp[t][g * PG], h, hx_tab[k], pbase,
                                      (double)(2 * w0 + 1) * h + hx_tab[0], tau <= kTauNC3, &are[lane * NS],
                                      &aim[lane * NS]);
                    } else {
                        auto &L = b32[0];
                        consume32<PG>(L.sc[t], L.Bk[t][k], &L.Cp[t][po], rf, r2f, r2d, sgl == 1, &fre[lane * NS],
                                      &fim[lane * NS], &tre[lane * NS], &tim[lane * NS]);
                    }
                }
            }
            if (!F64 || ++nb == kTileBatches) {
                nb = 0;
                for (int i = 0; i < 64 * NS; ++i) {
                    tre[i] += F64 ? are[i] : (double)fre[i];
                    tim[i] += F64 ? aim[i] : (double)fim[i];
                    are[i] = aim[i] = 0.0;
                    fre[i] = fim[i] = 0.0f;
                }
            }
        }
        for (int lane = 0; lane < 64; ++lane) {
            const int k = lane & 7, g = lane >> 3;
            const int po = lane >> 4, sgl = (lane >> 3) & 1;
            for (int slot = 0; slot < NS; ++slot) {
                const int i = lane * NS + slot;
                const double re = tre[i] + are[i];
                const double im = tim[i] + aim[i];
                const int p = F64 ? w0 + g * PG + slot / 2 : w0 + po + 4 * slot;
                const int sg = F64 ? slot % 2 : sgl;
                const double m = (double)(2 * p + 1) * h;
                const double r = sg == 0 ? m + hx_tab[k] : m - hx_tab[k];
                const int jn = sg == 0 ? kNH + k : kNH - 1 - k;
                const int64_t q = (int64_t)p * 16 + jn;
                out[2 * q] = re / (r * r);
                out[2 * q + 1] = im / (r * r);
            }
        }
    }
}

void build_tri_records(const double *verts, const int32_t *tris, int64_t nt, TriRec *rec);
#endif // HSD_TEST_HOOKS

} // namespace hsd

#ifdef HSD_TEST_HOOKS
extern "C" {

// mu^ at every node of a spherical product rule (n = 16 per panel, P a
// multiple of 8) through the wave kernel's producer/consumer bodies on the
// CPU (self checks only).  out[n_dir * P * 16 * 2].
int hsd__host_transform_wave(const double *verts, const int32_t *tris, int64_t nt, const double *dirs,
                             int64_t n_dir, const double *hx_tab, int P, double h, double tau, int form, double *out)
{
    using namespace hsd;
    if (P % 8 != 0) return -1;
    std::vector<TriRec> rec((size_t)nt);
    build_tri_records(verts, tris, nt, rec.data());
    const bool pg2 = P % 16 == 0;
    for (int64_t d = 0; d < n_dir; ++d) {
        double *o = out + 2 * d * (int64_t)P * 16;
        const double nx = dirs[3 * d], ny = dirs[3 * d + 1], nz = dirs[3 * d + 2];
        if (form == HSD_FORM_FP64) {
            if (pg2) host_wave_dir<2, true>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
            else host_wave_dir<1, true>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
        } else {
            if (pg2) host_wave_dir<2, false>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
            else host_wave_dir<1, false>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
        }
    }
    return 0;
}

} // extern "C"
#endif // HSD_TEST_HOOKS
