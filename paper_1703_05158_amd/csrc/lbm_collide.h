// Per-node collision of the D3Q19 step on gfx950, shared by the pull-collide
// kernel and the fused step kernel: moments (eqs. dens, momentum, with the
// Guo half-force velocity shift), the Smagorinsky relaxation time of
// Sec. 2.2, BGK collision with the Guo source (eq. Collision_step) and the
// store; and the inflow plane of Sec. 2.6 on the streamed populations.
#pragma once

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {
namespace dev {

// Inflow plane of a virtual cylinder (Sec. 2.6), on the streamed deviations
// g of a plane node: the directions from the removed domain (c_z = +1) were
// not received and keep the node's own values; with rho* the node's density,
// f_12 becomes rho - (rho* - f_12) for the cylinder density rho of this step
// (eq. ZIEBdesity9), u = sum f c / rho, and all populations are set to the
// equilibrium at (rho, u).  The collision then follows as at every node.
template <int S>
__device__ __forceinline__ void zieb_plane(const StepArgs &a, const typename Store<S>::T *src, uint32_t idx,
                                           float (&g)[kQ])
{
    using St = Store<S>;
    const size_t Ns = (size_t)a.Ns;
#pragma unroll
    for (int i = 1; i < kQ; ++i)
        if (CZ[i] == 1) g[i] = St::ld(at(src + (size_t)i * Ns, idx));
    const float rho = (float)a.zieb_state[0];
    float rd = 0.0f;
#pragma unroll
    for (int i = 0; i < kQ; ++i) rd += g[i];
    g[12] += rho - (a.rho0 + rd);  // deviations: f_12 - w_12 rho0 shifts by rho - rho*
    float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        jx += CX[i] * g[i];
        jy += CY[i] * g[i];
        jz += CZ[i] * g[i];
    }
    const float ir = 1.0f / rho;
    const float ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const float uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const float w = (float)wgt(i);
        const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        g[i] = w * (rho - a.rho0) + w * rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
    }
}

// c . v for a lattice vector c (components -1, 0, 1, compile-time) over its
// nonzero components only: a product with a zero component and a sum that
// starts from zero are operations the compiler may not drop (signed zeros,
// NaN), and here they would cost an instruction each.
__device__ __forceinline__ float cdot(int c0, int c1, int c2, float v0, float v1, float v2)
{
    float s = 0.0f;
    bool any = false;
    if (c0) {
        s = c0 > 0 ? v0 : -v0;
        any = true;
    }
    if (c1) {
        const float t = c1 > 0 ? v1 : -v1;
        s = any ? s + t : t;
        any = true;
    }
    if (c2) {
        const float t = c2 > 0 ? v2 : -v2;
        s = any ? s + t : t;
    }
    return s;
}

// s += t, where the first addition (first == true) takes t itself.
__device__ __forceinline__ void acc_first(float &s, bool &first, float t)
{
    s = first ? t : s + t;
    first = false;
}

// Collide the streamed deviations g of node idx and store the result into
// dst.  Every lane of the wavefront stores: a store with lanes switched off
// writes partial 128-byte lines, which cost a read-modify-write in HBM.  A
// solid lane (g = 0) stores the collision of the rest state, a finite value
// that nothing reads (a solid node's populations are never pulled, and a
// node that turns fluid is refilled).  `fluid` selects the lanes whose
// values count.
// kForce: the lattice has a body force (the Guo source and the half-force
// velocity shift); without one those terms are zero and are left out.
template <int S, bool kForce>
__device__ __forceinline__ void collide_store_f(const StepArgs &a, const float (&g)[kQ], bool fluid, uint32_t idx,
                                                typename Store<S>::T *__restrict__ dst)
{
    using St = Store<S>;
    const size_t Ns = (size_t)a.Ns;
    // moments in opposite pairs (i, i+9): even and odd parts
    float pe[10], po[10];
#pragma unroll
    for (int i = 1; i <= 9; ++i) {
        pe[i] = g[i] + g[i + 9];
        po[i] = g[i] - g[i + 9];
    }
    float rd = g[0], jx = 0.f, jy = 0.f, jz = 0.f;
    float sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, sxz = 0.f, syz = 0.f;
    bool fjx = true, fjy = true, fjz = true, fxx = true, fyy = true, fzz = true, fxy = true, fxz = true, fyz = true;
#pragma unroll
    for (int i = 1; i <= 9; ++i) {
        rd += pe[i];
        if (CX[i]) acc_first(jx, fjx, CX[i] > 0 ? po[i] : -po[i]);
        if (CY[i]) acc_first(jy, fjy, CY[i] > 0 ? po[i] : -po[i]);
        if (CZ[i]) acc_first(jz, fjz, CZ[i] > 0 ? po[i] : -po[i]);
        if (CX[i]) acc_first(sxx, fxx, pe[i]);
        if (CY[i]) acc_first(syy, fyy, pe[i]);
        if (CZ[i]) acc_first(szz, fzz, pe[i]);
        if (CX[i] * CY[i]) acc_first(sxy, fxy, CX[i] * CY[i] > 0 ? pe[i] : -pe[i]);
        if (CX[i] * CZ[i]) acc_first(sxz, fxz, CX[i] * CZ[i] > 0 ? pe[i] : -pe[i]);
        if (CY[i] * CZ[i]) acc_first(syz, fyz, CY[i] * CZ[i] > 0 ? pe[i] : -pe[i]);
    }
    const float rho = a.rho0 + rd;
    const float ir = __builtin_amdgcn_rcpf(rho);
    const float ux = (kForce ? jx + 0.5f * a.fx : jx) * ir;
    const float uy = (kForce ? jy + 0.5f * a.fy : jy) * ir;
    const float uz = (kForce ? jz + 0.5f * a.fz : jz) * ir;
    // second moment of f - feq
    const float third = 1.0f / 3.0f;
    const float pxx = sxx - rd * third - rho * ux * ux;
    const float pyy = syy - rd * third - rho * uy * uy;
    const float pzz = szz - rd * third - rho * uz * uz;
    const float pxy = sxy - rho * ux * uy;
    const float pxz = sxz - rho * ux * uz;
    const float pyz = syz - rho * uy * uz;
    // tau*: square roots by the hardware instruction (within 1 ulp), not
    // the correctly rounded sequence, which takes some fifteen instructions
    float tau;
    if (S == 0) {
        const float Qn = pxx * pxx + pyy * pyy + pzz * pzz + 2.0f * (pxy * pxy + pxz * pxz + pyz * pyz);
        tau = 0.5f * (a.tau0 + __builtin_amdgcn_sqrtf(a.tau0 * a.tau0 + a.smag_k * __builtin_amdgcn_sqrtf(Qn) * ir));
    } else {
        // 16-bit storage: the strain-rate norm accumulated in FP64; its
        // square root (of a sum of squares: well conditioned) and tau* in
        // FP32 like the rest
        const double Qn = (double)pxx * pxx + (double)pyy * pyy + (double)pzz * pzz +
                          2.0 * ((double)pxy * pxy + (double)pxz * pxz + (double)pyz * pyz);
        const float sq = __builtin_amdgcn_sqrtf((float)Qn);
        tau = 0.5f * (a.tau0 + __builtin_amdgcn_sqrtf(a.tau0 * a.tau0 + a.smag_k * sq * ir));
    }
    const float om = __builtin_amdgcn_rcpf(tau);
    const float om1 = 1.0f - om;
    const float cf = 1.0f - 0.5f * om;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = kForce ? ux * a.fx + uy * a.fy + uz * a.fz : 0.0f;
    if (a.flag && fluid && !(rho > 0.f && isfinite(uu))) atomicOr(a.flag, 1);
    // Post-collision deviation of direction i with weight w, for the pair
    // (i, i+9), c = c_i:
    //   equilibrium deviation  w (rd + rho (3 cu + 4.5 cu^2 - 1.5 uu)),
    //   Guo source             w cf (3 (c.F - u.F) + 9 cu c.F),
    // so om (feq - f) + source = w (A + cu (B cu + 9 cf cF)) +- w (3 om rho cu
    // + 3 cf cF) with A = om (rd - 1.5 rho uu) - 3 cf uF, B = 4.5 om rho; the
    // even part is shared by i and i+9, the odd part changes sign.  Factors
    // are taken per weight class (1/18 for the axis pairs, 1/36 for the
    // diagonal ones).
    const float A = kForce ? om * (rd - 1.5f * rho * uu) - 3.0f * cf * uF : om * (rd - 1.5f * rho * uu);
    const float B = 4.5f * om * rho, D = 3.0f * om * rho;
    const float w1 = (float)wgt(1), w2 = (float)wgt(4);
    const float a1 = w1 * A, a2 = w2 * A, b1 = w1 * B, b2 = w2 * B, d1 = w1 * D, d2 = w2 * D;
    const float e1 = 9.0f * w1 * cf, e2 = 9.0f * w2 * cf;   // times c.F: the source's cu term
    const float o1 = 3.0f * w1 * cf, o2 = 3.0f * w2 * cf;   // times c.F: the source's odd term
    St::stnt(at(dst, idx), om1 * g[0] + (float)wgt(0) * A);
#pragma unroll
    for (int i = 1; i <= 9; ++i) {
        const bool axis = wgt(i) == wgt(1);
        const float cu = cdot(CX[i], CY[i], CZ[i], ux, uy, uz);
        float ev, od;
        if (kForce) {
            const float cF = cdot(CX[i], CY[i], CZ[i], a.fx, a.fy, a.fz);
            ev = (axis ? a1 : a2) + cu * ((axis ? b1 : b2) * cu + (axis ? e1 : e2) * cF);
            od = (axis ? d1 : d2) * cu + (axis ? o1 : o2) * cF;
        } else {
            ev = (axis ? a1 : a2) + cu * ((axis ? b1 : b2) * cu);
            od = (axis ? d1 : d2) * cu;
        }
        const float vp = om1 * g[i] + (ev + od), vm = om1 * g[i + 9] + (ev - od);
        St::stnt(at(dst + (size_t)i * Ns, idx), vp);
        St::stnt(at(dst + (size_t)(i + 9) * Ns, idx), vm);
    }
}

template <int S>
__device__ __forceinline__ void collide_store(const StepArgs &a, const float (&g)[kQ], bool fluid, uint32_t idx,
                                              typename Store<S>::T *__restrict__ dst)
{
    if (a.fx != 0.0f || a.fy != 0.0f || a.fz != 0.0f)
        collide_store_f<S, true>(a, g, fluid, idx, dst);
    else
        collide_store_f<S, false>(a, g, fluid, idx, dst);
}

}  // namespace dev
}  // namespace lbm
