// Arithmetic of one cut lattice link (Sec. 2.3), shared by the boundary-link
// pass and the fused step kernel so that both give the same values bit for
// bit.  Contraction into fused multiply-adds is off here: the two kernels
// would otherwise be free to fuse different products.
//
// Notation: x is the fluid node, I the population it receives, K =
// opposite(I) the direction from x to the solid node p = x + c_K = x - c_I.
// Sphere links take q, the fraction of the link x -> p inside the fluid, and
// the wall velocity at x_b = x + q c_K; walls close their links at q = 1/2.
#pragma once

#include "lbm_device.h"

namespace lbm {
namespace dev {

// Sphere kinematics: centre in FP64, the rest in FP32.
struct SphereK {
    double X0, X1, X2;
    float V0, V1, V2, W0, W1, W2, R2;
};

__device__ __forceinline__ SphereK sphere_k(const double *B)
{
    SphereK k;
    k.X0 = B[0];
    k.X1 = B[1];
    k.X2 = B[2];
    k.V0 = (float)B[3];
    k.V1 = (float)B[4];
    k.V2 = (float)B[5];
    k.W0 = (float)B[6];
    k.W1 = (float)B[7];
    k.W2 = (float)B[8];
    k.R2 = (float)(B[9] * B[9]);
    return k;
}

// Geometry of the sphere link (x, I): the offset d = x - X (minimum image,
// FP64), the link fraction q and the moving-boundary term
// mw = w_K rho0 (c_I . u_w) with u_w = V + Omega x (x_b - X).
struct LinkGeo {
    double d0, d1, d2;
    float q, mw;
};

__device__ __forceinline__ LinkGeo link_geo(const SphereK &k, bool halfway, float rho0, int x, int y, int z, int nx,
                                            int ny, int nz, int I)
{
#pragma clang fp contract(off)
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);  // c_I = -c_K
    LinkGeo l;
    l.d0 = min_image((double)x - k.X0, nx);
    l.d1 = min_image((double)y - k.X1, ny);
    l.d2 = min_image((double)z - k.X2, nz);
    // the offset rounded once from FP64; q and the wall velocity in FP32
    const float e0 = (float)l.d0, e1 = (float)l.d1, e2 = (float)l.d2;
    if (halfway) {
        l.q = 0.5f;
    } else {
        // smallest root in (0, 1] of |d + q c_K|^2 = R^2, cancellation-free form
        const float bb = -(e0 * cx + e1 * cy + e2 * cz);
        const float aa = (float)(cx * cx + cy * cy + cz * cz);
        const float cc = (e0 * e0 + e1 * e1 + e2 * e2) - k.R2;
        const float disc = fmaxf(bb * bb - aa * cc, 0.0f);
        l.q = fminf(fmaxf(cc / (__builtin_sqrtf(disc) - bb), 0.0f), 1.0f);
    }
    // wall point x_b = x + q c_K relative to the centre, and its velocity
    const float f0 = e0 - l.q * cx, f1 = e1 - l.q * cy, f2 = e2 - l.q * cz;
    const float u0 = k.V0 + (k.W1 * f2 - k.W2 * f1);
    const float u1 = k.V1 + (k.W2 * f0 - k.W0 * f2);
    const float u2 = k.V2 + (k.W0 * f1 - k.W1 * f0);
    l.mw = (float)wgt(opp(I)) * rho0 * (cx * u0 + cy * u1 + cz * u2);
    return l;
}

// The population x receives along I across a sphere link (the two branches
// of Sec. 2.3 with the moving-boundary term): fk = P(x)[K], fa = P(x)[I],
// fb = P(x + c_I)[K] when the node behind x is fluid (behind), else unused.
__device__ __forceinline__ float link_value(float q, float fk, float fa, float fb, bool behind, float mw)
{
#pragma clang fp contract(off)
    if (q < 0.5f) return behind ? 2.0f * q * fk + (1.0f - 2.0f * q) * fb + 6.0f * mw : fk + 6.0f * mw;
    const float h = 0.5f / q;
    return h * fk + (1.0f - h) * fa + (3.0f / q) * mw;
}

// Moving-boundary term of a wall link (q = 1/2): 6 w_K rho0 (c_I . U).
__device__ __forceinline__ float wall_term(const double *wl, int I, float rho0)
{
#pragma clang fp contract(off)
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);
    return 6.0f * ((float)wgt(opp(I)) * rho0 * (float)(cx * wl[0] + cy * wl[1] + cz * wl[2]));
}

// Momentum handed to the body across the link, as full populations:
// P(x)[K] + f_I(x) + 2 w rho0 (the two stored deviations plus their
// weights), in FP64.
__device__ __forceinline__ double link_momentum(float fk, float vr, int I, float rho0)
{
#pragma clang fp contract(off)
    return (double)fk + (double)vr + 2.0 * wgt(I) * (double)rho0;
}

// Force mom c_K on the body and its torque arm x (F) about the lever arm
// (a0, a1, a2), added to acc[6] = {F, T}.
__device__ __forceinline__ void link_force(double mom, int I, double a0, double a1, double a2, double (&acc)[6])
{
#pragma clang fp contract(off)
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);
    const double F0 = -mom * cx, F1 = -mom * cy, F2 = -mom * cz;
    acc[0] += F0;
    acc[1] += F1;
    acc[2] += F2;
    acc[3] += a1 * F2 - a2 * F1;
    acc[4] += a2 * F0 - a0 * F2;
    acc[5] += a0 * F1 - a1 * F0;
}

// Lever arm of a sphere link: x_b - X = d - q c_I (FP64).
__device__ __forceinline__ void sphere_arm(const LinkGeo &l, int I, double &a0, double &a1, double &a2)
{
#pragma clang fp contract(off)
    const double qd = (double)l.q;
    a0 = l.d0 - qd * dcx(I);
    a1 = l.d1 - qd * dcy(I);
    a2 = l.d2 - qd * dcz(I);
}

// Lever arm of a wall link from node (x, y, z) about the wall's reference
// point: x + c_K / 2 - ref.
__device__ __forceinline__ void wall_arm(const double *wl, int I, int x, int y, int z, double &a0, double &a1,
                                         double &a2)
{
#pragma clang fp contract(off)
    a0 = (double)x - 0.5 * dcx(I) - wl[3];
    a1 = (double)y - 0.5 * dcy(I) - wl[4];
    a2 = (double)z - 0.5 * dcz(I) - wl[5];
}

// Exclusive prefix of `cnt` over the workgroup and the total (wtot: one int
// per wavefront in LDS).  Contains a barrier.
__device__ __forceinline__ int block_scan(int cnt, int *wtot, int &tot)
{
    constexpr int kWaves = kBlock / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int pos = incl - cnt;
    tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = wtot[w];
        if (w < wv) pos += t;
        tot += t;
    }
    return pos;
}

}  // namespace dev
}  // namespace lbm
