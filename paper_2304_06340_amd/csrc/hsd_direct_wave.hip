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
//     PG panels (2*PG nodes);
//   * FP64 form: per block of 32 triangles each lane computes the record of
//     one triangle and the direction (phase constants theta_mid, a/2, b/2,
//     closed-branch scale factors, series threshold and coefficients) into
//     LDS; then per batch of 4 triangles lane (t, jj) = (lane / 16,
//     lane % 16) computes, for triangle t, exp(-i h x_j c) (jj = j < 8, with
//     the series value of the wave's smallest radius with offset j) or the
//     panel-centre phases exp(-i m_p c) of the PG panels of group jj - 8, for
//     the three constants c;
//   * mixed form: per batch of 8 triangles lane (t, j) = (lane / 8, lane % 8)
//     computes the FP32 half-node phases of offset j and the panel-centre
//     phases of panels w0 + j + 8 q, and lane j = 0 the triangle's constants;
//   * consumer step: every lane forms its node phases by one complex product
//     per constant and node and accumulates, reading the batch from LDS.
//
// Per-lane sums use FP64 tiles of 32 triangles merged into running totals
// (the mixed form sums its closed branch in FP32 over a batch and adds that
// in FP64); K triangle splits on grid.y as in hsd_direct.hip.
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "hsd_internal.hpp"
#include "hsd_math.hpp"

namespace hsd {

namespace wv {

constexpr int kTB = 8;        // triangles per batch (mixed form)
constexpr int kNH = 8;        // node pairs per panel (16 GL nodes)
constexpr int kTB64 = 4;      // triangles per batch (FP64 form, 16 producer lanes each)
constexpr int kSB64 = 32;     // triangles per record block and tile sum (FP64 form)
constexpr double kGapFloor = 1e-150;
constexpr double kGapFloor32 = 1e-18;

// Per-(triangle, direction) constants.  ce/co are the coefficients of the
// divided-difference power series as a polynomial in the radius r:
// Re = sum_m ce[m] r^(2m), Im = r sum_m co[m] r^(2m) (see series_coefs).
// FP64 form: series through r^7; the first omitted term is below
// 9 G^8 / 10! of the leading 1/2, 1e-16 at the largest threshold the form
// accepts (G < 0.05) and 2.5e-22 at the default 0.01.  For thresholds up to
// kTauNC3 only the terms through r^5 are summed (first omitted term below
// 7 G^6 / 8! of the leading 1/2: 4e-15 at 0.015, 3.5e-16 at 0.01).
constexpr int kNC64 = 4;
constexpr double kTauNC3 = 0.015;
constexpr int kNC32 = (kMixedSeriesN + 1) / 2;  // through r^kMixedSeriesN (mixed form)
struct Scal32 { float rthr, Ka, Kb, c0lo; float ce[kNC32], co[kNC32]; };   // Ka, Kb, ce, co carry |J|

// FP64 form: one record per triangle of a block of kSB64, written by one lane
// each and read by the phase producers and consumers of the block's batches.
struct Rec64 {
    double tmid, ha, hb;          // phase constants theta_mid, a/2, b/2
    double ska, skb;              // sqrt(K_a), sqrt(K_b)
    double rthr, J, pad;          // series threshold tau / G, signed Jacobian
    double ce[kNC64], co[kNC64];  // carry |J|
    double pad2[2];               // 144 B: the 16-byte units of 16 consecutive records fall in distinct LDS banks
};
struct Ser64 { double y, x; };    // r^2-scaled series value (Re, Im) at one radius
template <int PG> struct Batch64 {
    cs64 Bk[kTB64][kNH][3];
    cs64 Cp[kTB64][kNH * PG][3];
    Ser64 S1[kTB64][kNH];         // series value of slot (panel w0, minus) per node offset
};
template <int PG> struct Lds64 {
    Rec64 rec[kSB64];
    Batch64<PG> b;
};
// Mixed form: record of a triangle and direction, one per triangle of a
// block of kSB64 as in the FP64 form; the phase constants stay FP64 (the
// phases are reduced in FP64).
struct Rec32 {
    double tmid, ha, hb;          // phase constants theta_mid, a/2, b/2
    float sgn, pad;               // sign of J
    Scal32 sc;
};
template <int PG> struct Batch32 {
    cs32 Bk[kTB][kNH][3];
    cs32 Cp[kTB][kNH * PG][3];
};
template <int PG> struct Lds32 {
    Rec32 rec[kSB64];
    Batch32<PG> b;
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

// Phase e^{-i h c} of the first panel's centre, held by lane 8 of each group
// of 16 producer lanes (one triangle) when the wave starts at panel 0:
// broadcast within the group by a DPP row broadcast (row_newbcast:8, every
// lane reads lane 8 of its row of 16; a VALU move, no LDS access).  The host
// emulation recomputes what that lane computed.
HSD_HD cs64 group_first_phase(cs64 own, double hc, const cs64 *turn)
{
#if defined(__HIP_DEVICE_COMPILE__)
    (void)hc;
    (void)turn;
    cs64 r;
    r.c = __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(own.c), 0x158, 0xf, 0xf, false),
                           __builtin_amdgcn_mov_dpp(__double2loint(own.c), 0x158, 0xf, 0xf, false));
    r.s = __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(own.s), 0x158, 0xf, 0xf, false),
                           __builtin_amdgcn_mov_dpp(__double2loint(own.s), 0x158, 0xf, 0xf, false));
    return r;
#else
    (void)own;
    return sincos64_tab(hc, turn);
#endif
}

// Record of a triangle and direction (FP64 form), computed once per pair by
// one lane.  The closed branch needs K_a sin^2(r a/2), K_a sin(r a/2)
// cos(r a/2) and the same for b, with K_a = 2 |J| / (G a), K_b = 2 |J| /
// (G b); their square roots go onto the half-gap phases (see produce64).
HSD_HD Rec64 make_rec64(const TriDir &td, double tau)
{
    Rec64 R;
    R.tmid = td.tmid;
    R.ha = 0.5 * td.ac;
    R.hb = 0.5 * td.bc;
    // 1/ac and 1/bc from one reciprocal of ac bc (both gaps are floored at
    // 1e-150, so the product stays a normal number)
    const double aJ = fabs(td.J);
    const double rab = rcp64(td.ac * td.bc);
    const double t = 2.0 * aJ * td.iG;
    R.ska = sqrt_pos64(t * (td.bc * rab));
    R.skb = sqrt_pos64(t * (td.ac * rab));
    R.rthr = tau * td.iG;
    R.J = td.J;
    R.pad = 0.0;
    R.pad2[0] = R.pad2[1] = 0.0;
    series_coefs<kNC64>(td.ac, td.bc, aJ, R.ce, R.co);
    return R;
}

// Record of a block that a lane computes: lane % kSB64, always in
// [0, kSB64); the lanes below kSB64 write theirs, the others compute a copy.
HSD_HD int rec_of_lane(int lane) { return lane % kSB64; }

// Series value (Re, Im, both times r^2) at radius r from a record.
HSD_HD Ser64 series_at(const Rec64 &R, double r, bool nc3)
{
    const double r2 = r * r;
    double pe, po;
    if (nc3)
        series_eval<3>(R.ce, R.co, r2, pe, po);
    else
        series_eval<kNC64>(R.ce, R.co, r2, pe, po);
    return Ser64{r2 * pe, r2 * r * po};
}

// Phase producer, FP64: lane (t, jj) = (lane / 16, lane % 16) of a batch of
// kTB64 triangles, one phase per constant c = theta_mid, a/2, b/2.
//   jj < 8: the half-node phases exp(-i h x_j c) of node offset j = jj, with
//     the sign of J on the theta_mid one and sqrt(K_a), sqrt(K_b) on the two
//     half-gap ones (the consumer's phase products then give sqrt(K)
//     e^{-i r g/2}, and the closed branch's four terms are two squares and
//     two products of their parts); and the series value of the wave's
//     smallest-radius slot with that offset (panel w0, radius (2 w0 + 1) h -
//     h x_j), taken by the consumers where that radius is below the
//     threshold;
//   jj >= 8: the panel-centre phases exp(-i m_p c) of panels w0 + j PG + q,
//     j = jj - 8.  ONE (the wave covers all panels of its direction, w0 = 0):
//     the second panel's phase is the first one's times e^{-2 i h c}, the
//     square of the phase of the first panel's centre, which lane jj = 8
//     holds.
template <int PG, bool ONE>
HSD_HD void produce64(const Rec64 &rec, double h, const double *hx_tab, int jj, int w0, bool nc3,
                      const cs64 *turn, cs64 Bk[3], cs64 (*Cp)[3], Ser64 *s1)
{
    // The whole record is read up front and every lane runs the same
    // arithmetic (a half-node lane's factors on the phases, 1 for a
    // panel-centre lane), so the role only picks where the results go.
    const Rec64 R = rec;
    const bool half = jj < kNH;
    const int j = jj & (kNH - 1);
    const double hxj = hx_tab[j];
    const double mult = half ? hxj : (double)(2 * (w0 + j * PG) + 1) * h;
    const double fr[3] = {R.tmid, R.ha, R.hb};
    const double fac[3] = {half && R.J < 0.0 ? -1.0 : 1.0, half ? R.ska : 1.0, half ? R.skb : 1.0};
    cs64 ph[3], step[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ph[c] = sincos64_tab(mult * fr[c], turn);
    if constexpr (ONE && PG > 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cs64 e1 = group_first_phase(ph[c], h * fr[c], turn);
            step[c] = pmul(e1, e1);
        }
    }
    const Ser64 sv = series_at(R, (double)(2 * w0 + 1) * h - hxj, nc3);
    cs64 *dst = half ? Bk : Cp[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c] = cs64{fac[c] * ph[c].c, fac[c] * ph[c].s};
    if (half) {
        *s1 = sv;
    } else {
#pragma unroll
        for (int q = 1; q < PG; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (ONE)
                    ph[c] = pmul(ph[c], step[c]);
                else
                    ph[c] = sincos64_tab((double)(2 * (w0 + j * PG + q) + 1) * h * fr[c], turn);
                Cp[q][c] = ph[c];
            }
        }
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
// h x_0).  While the triangle's threshold is not above r_others, only that
// slot of the lanes of the first panel group (radius (2 w0 + 1) h - h x_k)
// can be below it, and those lanes take the series value the producer
// stored (s1); otherwise every slot compares and evaluates the series from
// the record.  nc3: thresholds up to kTauNC3, series through r^5.
template <int PG>
HSD_HD void consume64(const Rec64 &R, const cs64 Bk[3], const cs64 (*Cp)[3], const Ser64 &s1, double h,
                      double hx, int pbase, double r_others, bool nc3, double *acc_re, double *acc_im)
{
    constexpr int NS = 2 * PG;
    const double rthr = R.rthr;
    const Ser64 sv = s1;
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
    // the stored series value is taken without a branch; where it does not
    // belong to this slot (a later panel group) the triangle takes the
    // compare-every-slot path below, which overwrites it
    const bool take = rs[1] < rthr;
    Yr[1] = take ? sv.y : Yr[1];
    Xr[1] = take ? sv.x : Xr[1];
    if (rthr > r_others) {
#pragma unroll
        for (int slot = 0; slot < NS; ++slot) {
            if (rs[slot] < rthr) {
                const Ser64 v = series_at(R, rs[slot], nc3);
                Yr[slot] = v.y;
                Xr[slot] = v.x;
            }
        }
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
HSD_HD Rec32 make_rec32(const TriDir &td, double tau)
{
    Rec32 R;
    R.tmid = td.tmid;
    R.ha = 0.5 * td.ac;
    R.hb = 0.5 * td.bc;
    R.sgn = td.J < 0.0 ? -1.0f : 1.0f;
    R.pad = 0.0f;
    const double aJ = fabs(td.J);
    const double rab = rcp64(td.ac * td.bc);   // gaps floored at 1e-18
    const double t = 2.0 * aJ * td.iG;
    R.sc.Ka = (float)(t * (td.bc * rab));
    R.sc.Kb = (float)(t * (td.ac * rab));
    R.sc.rthr = (float)(fmax(tau, kMixedTau) * td.iG);   // decides the branch only
    double ce[kNC32], co[kNC32];
    series_coefs<kNC32>(td.ac, td.bc, aJ, ce, co);
    R.sc.ce[0] = (float)ce[0];
    R.sc.c0lo = (float)(ce[0] - (double)R.sc.ce[0]);
#pragma unroll
    for (int m = 1; m < kNC32; ++m) R.sc.ce[m] = (float)ce[m];
#pragma unroll
    for (int m = 0; m < kNC32; ++m) R.sc.co[m] = (float)co[m];
    return R;
}

// Part j of a triangle's phases (mixed form), from its record.
template <int PG>
HSD_HD void produce32(const Rec32 &rec, double h, const double *hx_tab, int j, int w0, cs32 Bk[3], cs32 (*Cp)[3])
{
    const double fr[3] = {rec.tmid, rec.ha, rec.hb};
    const double hx = hx_tab[j];
    const float sgn = rec.sgn;
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
// kernel bodies: 4 waves per block, one direction (and panel window) per wave
// ---------------------------------------------------------------------------

// Slot -> output node: panel p, sign sg (0: m_p + h x_k), r^2 divided out.
__device__ __forceinline__ void store_slot(double2 *out, int p, int sg, int k, double h, double hx, double re,
                                           double im)
{
    const double m = (double)(2 * p + 1) * h;
    const double r = sg == 0 ? m + hx : m - hx;
    const double inv = 1.0 / (r * r);
    const int jn = sg == 0 ? wv::kNH + k : wv::kNH - 1 - k;
    out[(int64_t)p * (2 * wv::kNH) + jn] = make_double2(re * inv, im * inv);
}

// FP64 form.  Per block of kSB64 triangles: lane l < kSB64 writes the record
// of triangle l; then per batch of kTB64 triangles the 64 lanes produce the
// phases (produce64) and every lane consumes the batch (consume64).  The
// lane's slots are summed in FP64 over the block (a tile of kSB64
// triangles) and merged into the running totals after it.
template <int PG, bool ONE>
__device__ __forceinline__ void direct_wave_body64(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    using namespace wv;
    constexpr int NS = 2 * PG;
    __shared__ Lds64<PG> lds[4];
    __shared__ cs64 turn[32];     // e^{i k pi/16} for the FP64 sin/cos
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x < 32) turn[threadIdx.x] = turn16((int)threadIdx.x);
    __syncthreads();
    const int wpd = P / (kNH * PG);                 // waves per direction
    const int64_t gw = (int64_t)blockIdx.x * 4 + w;
    const bool valid = gw < d_count * wpd;
    const int64_t GW = valid ? gw : 0;
    const int64_t d = d_begin + GW / wpd;
    const int w0 = (int)(GW % wpd) * kNH * PG;       // first panel of the wave
    const double nx = dirs[3 * d], ny = dirs[3 * d + 1], nz = dirs[3 * d + 2];
    const int k = lane & 7, g = lane >> 3;             // consumer roles
    const int pt = lane >> 4, pj = lane & 15;          // phase producer roles
    const double hx = hx_tab[k];
    const int pbase = w0 + g * PG;                     // slots (pl, sg): panel pbase + pl
    const double r_others = (double)(2 * w0 + 1) * h + hx_tab[0];   // see consume64
    const bool nc3 = tau <= kTauNC3;
    auto &L = lds[w];

    const int64_t ntot = nA + nB;
    const int K = gridDim.y;
    const int64_t t_begin = ntot * blockIdx.y / K;
    const int64_t t_end = ntot * (blockIdx.y + 1) / K;

    double tot_re[NS], tot_im[NS], acc_re[NS], acc_im[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) { tot_re[i] = 0.0; tot_im[i] = 0.0; acc_re[i] = 0.0; acc_im[i] = 0.0; }

    for (int64_t sb = t_begin; sb < t_end; sb += kSB64) {
        const int nsb = (int)((t_end - sb) < kSB64 ? (t_end - sb) : kSB64);
        {   // records (lanes l and l + 32 compute the same one)
            const int l = rec_of_lane(lane);
            double J;
            const TriRec *rp = wv::tri_at(A, nA, B, sb + (l < nsb ? l : 0), J);
            const Rec64 R = make_rec64(tri_dir(*rp, J, nx, ny, nz, kGapFloor), tau);
            if (lane < kSB64) L.rec[l] = R;
        }
        wave_lds_sync();
        for (int b0 = 0; b0 < nsb; b0 += kTB64) {
            const int nvalid = (nsb - b0) < kTB64 ? (nsb - b0) : kTB64;
            const int j = pj & (kNH - 1);
            produce64<PG, ONE>(L.rec[b0 + (pt < nvalid ? pt : 0)], h, hx_tab, pj, w0, nc3, turn, L.b.Bk[pt][j],
                               &L.b.Cp[pt][j * PG], &L.b.S1[pt][j]);
            wave_lds_sync();
#pragma unroll
            for (int t = 0; t < kTB64; ++t)   // unrolled: the batch offsets become immediates
                if (t < nvalid)
                    consume64<PG>(L.rec[b0 + t], L.b.Bk[t][k], &L.b.Cp[t][g * PG], L.b.S1[t][k], h, hx, pbase,
                                  r_others, nc3, acc_re, acc_im);
            wave_lds_sync();
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            tot_re[i] += acc_re[i];
            tot_im[i] += acc_im[i];
            acc_re[i] = 0.0;
            acc_im[i] = 0.0;
        }
    }
    if (!valid) return;
    double2 *out = partial + (int64_t)blockIdx.y * N + d * (int64_t)(P * 2 * kNH);
#pragma unroll
    for (int slot = 0; slot < NS; ++slot)
        store_slot(out, pbase + slot / 2, slot % 2, k, h, hx, tot_re[slot], tot_im[slot]);
}

// Mixed form: per block of kSB64 triangles lane l < kSB64 writes the record
// of triangle l; then per batch of kTB triangles lane (t, j) = (lane / 8,
// lane % 8) produces part j of triangle t (produce32); the closed branch's
// FP32 sums over one batch are flushed into the FP64 running totals after
// every batch (the series branch adds to the running totals directly, see
// consume32).
template <int PG>
__device__ __forceinline__ void direct_wave_body32(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    using namespace wv;
    constexpr int NS = 2 * PG;
    __shared__ Lds32<PG> lds[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wpd = P / (kNH * PG);                 // waves per direction
    const int64_t gw = (int64_t)blockIdx.x * 4 + w;
    const bool valid = gw < d_count * wpd;
    const int64_t GW = valid ? gw : 0;
    const int64_t d = d_begin + GW / wpd;
    const int w0 = (int)(GW % wpd) * kNH * PG;       // first panel of the wave
    const double nx = dirs[3 * d], ny = dirs[3 * d + 1], nz = dirs[3 * d + 2];
    const int k = lane & 7;
    const int pt = lane >> 3, pj = lane & 7;           // producer roles
    const double hx = hx_tab[k];
    // lanes are laid out as (po, sg, k), see consume32
    const int po = lane >> 4, sgl = (lane >> 3) & 1;
    float rf[NS], r2f[NS];
    double r2d[NS];
    mixed_lane_radii<PG>(w0, po, sgl, h, hx, rf, r2f, r2d);
    auto &L = lds[w];

    const int64_t ntot = nA + nB;
    const int K = gridDim.y;
    const int64_t t_begin = ntot * blockIdx.y / K;
    const int64_t t_end = ntot * (blockIdx.y + 1) / K;

    double tot_re[NS], tot_im[NS];
    float acc_re[NS], acc_im[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) { tot_re[i] = 0.0; tot_im[i] = 0.0; acc_re[i] = 0.0f; acc_im[i] = 0.0f; }

    for (int64_t sb = t_begin; sb < t_end; sb += kSB64) {
        const int nsb = (int)((t_end - sb) < kSB64 ? (t_end - sb) : kSB64);
        {   // records (lanes l and l + 32 compute the same one)
            const int l = rec_of_lane(lane);
            double J;
            const TriRec *rp = wv::tri_at(A, nA, B, sb + (l < nsb ? l : 0), J);
            const Rec32 R = make_rec32(tri_dir(*rp, J, nx, ny, nz, kGapFloor32), tau);
            if (lane < kSB64) L.rec[l] = R;
        }
        wave_lds_sync();
        for (int b0 = 0; b0 < nsb; b0 += kTB) {
            const int nvalid = (nsb - b0) < kTB ? (nsb - b0) : kTB;
            produce32<PG>(L.rec[b0 + (pt < nvalid ? pt : 0)], h, hx_tab, pj, w0, L.b.Bk[pt][pj], L.b.Cp[pt]);
            wave_lds_sync();
            for (int t = 0; t < nvalid; ++t)
                consume32<PG>(L.rec[b0 + t].sc, L.b.Bk[t][k], &L.b.Cp[t][po], rf, r2f, r2d, sgl == 1, acc_re, acc_im,
                              tot_re, tot_im);
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                tot_re[i] += (double)acc_re[i];
                tot_im[i] += (double)acc_im[i];
                acc_re[i] = 0.0f;
                acc_im[i] = 0.0f;
            }
        }
    }
    if (!valid) return;
    double2 *out = partial + (int64_t)blockIdx.y * N + d * (int64_t)(P * 2 * kNH);
#pragma unroll
    for (int slot = 0; slot < NS; ++slot)   // slot -> panel w0 + po + 4 slot, sign sgl
        store_slot(out, w0 + po + 4 * slot, sgl, k, h, hx, tot_re[slot], tot_im[slot]);
}

// FP64 form: its LDS (9.5 KB per wave: 32 records and one batch, 38.5 KB per
// block) allows 4 blocks per CU.  ONE: one wave per direction (the wave
// starts at panel 0).
template <int PG, bool ONE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_direct_wave(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    direct_wave_body64<PG, ONE>(A, nA, B, nB, dirs, hx_tab, d_begin, d_count, P, h, tau, N, partial);
}

// Mixed form: 7.5 KB of LDS per wave (32 records and one batch of 8
// triangles, 30 KB per block) allow 5 blocks per CU; held to 5 waves per
// SIMD (96 VGPRs, a few spills at the record-block level, none in the batch
// loops): 2% faster than at 4.
template <int PG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_direct_wave_mixed(
    const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
    const double *__restrict__ dirs, const double *__restrict__ hx_tab, int64_t d_begin, int64_t d_count,
    int P, double h, double tau, int64_t N, double2 *__restrict__ partial)
{
    direct_wave_body32<PG>(A, nA, B, nB, dirs, hx_tab, d_begin, d_count, P, h, tau, N, partial);
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
// Slot of a lane -> output node (as store_slot).
static void host_store(double *out, int p, int sg, int k, double h, const double *hx_tab, double re, double im)
{
    const double m = (double)(2 * p + 1) * h;
    const double r = sg == 0 ? m + hx_tab[k] : m - hx_tab[k];
    const int jn = sg == 0 ? wv::kNH + k : wv::kNH - 1 - k;
    const int64_t q = (int64_t)p * 16 + jn;
    out[2 * q] = re / (r * r);
    out[2 * q + 1] = im / (r * r);
}

template <int PG>
static void host_wave_dir64(const TriRec *A, int64_t nA, double nx, double ny, double nz, const double *hx_tab,
                            int P, double h, double tau, double *out /* [P*16*2] */)
{
    using namespace wv;
    constexpr int NS = 2 * PG;
    const int wpd = P / (kNH * PG);
    const bool nc3 = tau <= kTauNC3;
    std::vector<Lds64<PG>> lv(1);
    auto &L = lv[0];
    cs64 turn[32];
    for (int k = 0; k < 32; ++k) turn[k] = turn16(k);
    for (int wi = 0; wi < wpd; ++wi) {
        const int w0 = wi * kNH * PG;
        const double r_others = (double)(2 * w0 + 1) * h + hx_tab[0];
        std::vector<double> tre(64 * NS, 0.0), tim(64 * NS, 0.0), are(64 * NS, 0.0), aim(64 * NS, 0.0);
        for (int64_t sb = 0; sb < nA; sb += kSB64) {
            const int nsb = (int)std::min<int64_t>(kSB64, nA - sb);
            for (int lane = 0; lane < 64; ++lane) {   // as the device lanes, with a bounds check
                const int l = rec_of_lane(lane);
                const int64_t gi = sb + (l < nsb ? l : 0);
                if (l < 0 || l >= kSB64 || gi < 0 || gi >= nA) std::abort();
                double J;
                const TriRec *rp = wv::tri_at(A, nA, nullptr, gi, J);
                const Rec64 R = make_rec64(tri_dir(*rp, J, nx, ny, nz, kGapFloor), tau);
                if (lane < kSB64) L.rec[l] = R;
            }
            for (int b0 = 0; b0 < nsb; b0 += kTB64) {
                const int nvalid = std::min(kTB64, nsb - b0);
                for (int lane = 0; lane < 64; ++lane) {
                    const int pt = lane >> 4, pj = lane & 15, j = pj & (kNH - 1);
                    const Rec64 &R = L.rec[b0 + (pt < nvalid ? pt : 0)];
                    if (wpd == 1)
                        produce64<PG, true>(R, h, hx_tab, pj, w0, nc3, turn, L.b.Bk[pt][j], &L.b.Cp[pt][j * PG],
                                            &L.b.S1[pt][j]);
                    else
                        produce64<PG, false>(R, h, hx_tab, pj, w0, nc3, turn, L.b.Bk[pt][j], &L.b.Cp[pt][j * PG],
                                             &L.b.S1[pt][j]);
                }
                for (int lane = 0; lane < 64; ++lane) {
                    const int k = lane & 7, g = lane >> 3;
                    for (int t = 0; t < nvalid; ++t)
                        consume64<PG>(L.rec[b0 + t], L.b.Bk[t][k], &L.b.Cp[t][g * PG], L.b.S1[t][k], h, hx_tab[k],
                                      w0 + g * PG, r_others, nc3, &are[lane * NS], &aim[lane * NS]);
                }
            }
            for (int i = 0; i < 64 * NS; ++i) {
                tre[i] += are[i];
                tim[i] += aim[i];
                are[i] = aim[i] = 0.0;
            }
        }
        for (int lane = 0; lane < 64; ++lane) {
            const int k = lane & 7, g = lane >> 3;
            for (int slot = 0; slot < NS; ++slot)
                host_store(out, w0 + g * PG + slot / 2, slot % 2, k, h, hx_tab, tre[lane * NS + slot],
                           tim[lane * NS + slot]);
        }
    }
}

template <int PG>
static void host_wave_dir32(const TriRec *A, int64_t nA, double nx, double ny, double nz, const double *hx_tab,
                            int P, double h, double tau, double *out /* [P*16*2] */)
{
    using namespace wv;
    constexpr int NS = 2 * PG;
    const int wpd = P / (kNH * PG);
    std::vector<Lds32<PG>> lv(1);
    auto &L = lv[0];
    for (int wi = 0; wi < wpd; ++wi) {
        const int w0 = wi * kNH * PG;
        std::vector<double> tre(64 * NS, 0.0), tim(64 * NS, 0.0);
        std::vector<float> fre(64 * NS, 0.0f), fim(64 * NS, 0.0f);
        for (int64_t sb = 0; sb < nA; sb += kSB64) {
            const int nsb = (int)std::min<int64_t>(kSB64, nA - sb);
            for (int lane = 0; lane < 64; ++lane) {   // as the device lanes, with a bounds check
                const int l = rec_of_lane(lane);
                const int64_t gi = sb + (l < nsb ? l : 0);
                if (l < 0 || l >= kSB64 || gi < 0 || gi >= nA) std::abort();
                double J;
                const TriRec *rp = wv::tri_at(A, nA, nullptr, gi, J);
                const Rec32 R = make_rec32(tri_dir(*rp, J, nx, ny, nz, kGapFloor32), tau);
                if (lane < kSB64) L.rec[l] = R;
            }
            for (int b0 = 0; b0 < nsb; b0 += kTB) {
                const int nvalid = std::min(kTB, nsb - b0);
                for (int lane = 0; lane < 64; ++lane) {
                    const int pt = lane >> 3, pj = lane & 7;
                    produce32<PG>(L.rec[b0 + (pt < nvalid ? pt : 0)], h, hx_tab, pj, w0, L.b.Bk[pt][pj], L.b.Cp[pt]);
                }
                for (int lane = 0; lane < 64; ++lane) {
                    const int k = lane & 7;
                    const int po = lane >> 4, sgl = (lane >> 3) & 1;
                    float rf[NS], r2f[NS];
                    double r2d[NS];
                    mixed_lane_radii<PG>(w0, po, sgl, h, hx_tab[k], rf, r2f, r2d);
                    for (int t = 0; t < nvalid; ++t)
                        consume32<PG>(L.rec[b0 + t].sc, L.b.Bk[t][k], &L.b.Cp[t][po], rf, r2f, r2d, sgl == 1,
                                      &fre[lane * NS], &fim[lane * NS], &tre[lane * NS], &tim[lane * NS]);
                }
                for (int i = 0; i < 64 * NS; ++i) {
                    tre[i] += (double)fre[i];
                    tim[i] += (double)fim[i];
                    fre[i] = fim[i] = 0.0f;
                }
            }
        }
        for (int lane = 0; lane < 64; ++lane) {
            const int k = lane & 7;
            const int po = lane >> 4, sgl = (lane >> 3) & 1;
            for (int slot = 0; slot < NS; ++slot)
                host_store(out, w0 + po + 4 * slot, sgl, k, h, hx_tab, tre[lane * NS + slot], tim[lane * NS + slot]);
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
            if (pg2) host_wave_dir64<2>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
            else host_wave_dir64<1>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
        } else {
            if (pg2) host_wave_dir32<2>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
            else host_wave_dir32<1>(rec.data(), nt, nx, ny, nz, hx_tab, P, h, tau, o);
        }
    }
    return 0;
}

} // extern "C"
#endif // HSD_TEST_HOOKS
