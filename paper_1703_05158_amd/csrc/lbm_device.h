// Device-side helpers shared by the gfx950 kernels: the D3Q19 tables of the
// paper's Table 1, population storage formats, index arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {
namespace dev {

// Table 1: c_i for i = 0..18.
constexpr int CX[kQ] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
constexpr int CY[kQ] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
constexpr int CZ[kQ] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};

constexpr uint64_t pack_dir(const int (&c)[kQ])
{
    uint64_t v = 0;
    for (int i = 0; i < kQ; ++i) v |= (uint64_t)(c[i] + 1) << (2 * i);
    return v;
}
constexpr uint64_t kPX = pack_dir(CX), kPY = pack_dir(CY), kPZ = pack_dir(CZ);

// Runtime-indexed lookups (cold paths) without memory traffic.
__device__ __forceinline__ int dcx(int i) { return (int)((kPX >> (2 * i)) & 3) - 1; }
__device__ __forceinline__ int dcy(int i) { return (int)((kPY >> (2 * i)) & 3) - 1; }
__device__ __forceinline__ int dcz(int i) { return (int)((kPZ >> (2 * i)) & 3) - 1; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }

// Weights: w0 = 1/3, axis directions (1,2,3,10,11,12) 1/18, others 1/36.
__host__ __device__ constexpr double wgt(int i)
{
    return i == 0 ? 1.0 / 3.0 : (((0x1C0Eu >> i) & 1u) ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Storage of deviations g = f - w rho0.  stnt is the store of the step
// kernel's output: a non-temporal hint, since the whole next state streams
// through the caches before any of it is read again.
template <int S> struct Store;
template <> struct Store<0> {
    using T = float;
    static __device__ __forceinline__ float cvt(T v) { return v; }  // a stored value as FP32
    static __device__ __forceinline__ float ld(const T *p) { return *p; }
    static __device__ __forceinline__ void st(T *p, float v) { *p = v; }
    static __device__ __forceinline__ void stnt(T *p, float v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ float round(float v) { return v; }
    // a stored value as the 32-bit word a load into LDS leaves (16-bit
    // values zero-extended), and back
    static __device__ __forceinline__ float from_bits(uint32_t w) { return __uint_as_float(w); }
    static __device__ __forceinline__ uint32_t to_bits(float v) { return __float_as_uint(v); }
};
template <> struct Store<1> {
    using T = _Float16;
    static __device__ __forceinline__ float cvt(T v) { return (float)v; }
    static __device__ __forceinline__ float ld(const T *p) { return (float)*p; }
    static __device__ __forceinline__ void st(T *p, float v) { *p = (_Float16)v; }
    static __device__ __forceinline__ void stnt(T *p, float v) { __builtin_nontemporal_store((_Float16)v, p); }
    static __device__ __forceinline__ float round(float v) { return (float)(_Float16)v; }
    static __device__ __forceinline__ float from_bits(uint32_t w)
    {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)w);
    }
    static __device__ __forceinline__ uint32_t to_bits(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};
template <> struct Store<2> {  // bfloat16 as raw bits, round to nearest even
    using T = uint16_t;
    static __device__ __forceinline__ float cvt(T v) { return __uint_as_float((uint32_t)v << 16); }
    static __device__ __forceinline__ float ld(const T *p) { return __uint_as_float((uint32_t)*p << 16); }
    // gfx950's conversion instruction (v_cvt_pk_bf16_f32) rounds to nearest
    // even: one instruction where the rounding in integer arithmetic takes six
    static __device__ __forceinline__ uint16_t bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    static __device__ __forceinline__ void st(T *p, float v) { *p = bits(v); }
    static __device__ __forceinline__ void stnt(T *p, float v) { __builtin_nontemporal_store(bits(v), p); }
    static __device__ __forceinline__ float round(float v) { return __uint_as_float((uint32_t)bits(v) << 16); }
    static __device__ __forceinline__ float from_bits(uint32_t w) { return __uint_as_float(w << 16); }
    static __device__ __forceinline__ uint32_t to_bits(float v) { return bits(v); }
};

// Element `e` of an array whose byte size fits in 32 bits: the offset is a
// zero-extended 32-bit value, so the load can use a uniform base register.
template <typename T>
__device__ __forceinline__ const T *at(const T *base, uint32_t e)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint64_t)(e * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T *at(T *base, uint32_t e)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (uint64_t)(e * (uint32_t)sizeof(T)));
}

__device__ __forceinline__ int wrap_add(int a, int d, int n)
{
    const int r = a + d;
    return r < 0 ? r + n : (r >= n ? r - n : r);
}

// Workgroups go round-robin over the 8 XCDs.  The work items are handed out
// in chunks of kXcdChunk consecutive items, chunk c to XCD c mod 8, so that
// neighbouring items share an L2 while every XCD draws from the whole range
// (a contiguous eighth per XCD loads the XCDs unevenly wherever the work is
// not spread evenly over the range).  Item i of XCD x's share, in order:
constexpr int kXcdChunk = 64;

__device__ __forceinline__ int xcd_item(int x, int i) { return ((i / kXcdChunk) * 8 + x) * kXcdChunk + i % kXcdChunk; }

__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int full = nblocks / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (b >= full) return b;  // the last partial round in plain order
    return xcd_item(b & 7, b >> 3);
}

// A copy of v that the compiler knows to be the same in every lane (the
// value of the first active lane), so that it can live in scalar registers:
// for argument blocks that a kernel loads from memory (the batch kernels).
template <typename T>
__device__ __forceinline__ T uniform(const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}

// Wrap a coordinate known to lie in [-n, 2n).
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

// A sphere the rasteriser accepts: radius in (0, min(n)/2 - 1), centre in the box.
__device__ __forceinline__ bool body_ok(const double *B, int nx, int ny, int nz)
{
    const double lim = 0.5 * (double)min(nx, min(ny, nz)) - 1.0;
    return B[9] > 0.0 && B[9] < lim && B[0] >= 0.0 && B[0] < nx && B[1] >= 0.0 && B[1] < ny &&
           B[2] >= 0.0 && B[2] < nz;
}

// Deviation of the equilibrium at rho0 and velocity u from the rest state:
// w_i rho0 (3 c.u + 4.5 (c.u)^2 - 1.5 u.u).
__device__ __forceinline__ double eq_dev(int i, double rho0, double u0, double u1, double u2)
{
    const double cu = dcx(i) * u0 + dcy(i) * u1 + dcz(i) * u2;
    return wgt(i) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * (u0 * u0 + u1 * u1 + u2 * u2));
}

// |p - X|^2 with the minimum image, as a plain product-sum evaluated left to
// right without fused multiply-add (the owner test compares it with R^2).
// The products and sums are written here, under contraction off: the
// compiler would otherwise fuse them into FMAs (as it does with __dmul_rn and
// __dadd_rn, which are ordinary operations in device code), and a node
// exactly on a sphere's surface would be decided differently.
__device__ __forceinline__ double dist2(const double *B, int px, int py, int pz, int nx, int ny, int nz)
{
#pragma clang fp contract(off)
    const double dx = min_image((double)px - B[0], nx);
    const double dy = min_image((double)py - B[1], ny);
    const double dz = min_image((double)pz - B[2], nz);
    const double sxy = dx * dx + dy * dy;
    return sxy + dz * dz;
}

__device__ __forceinline__ bool inside(const double *B, int px, int py, int pz, int nx, int ny, int nz)
{
#pragma clang fp contract(off)
    const double r2 = B[9] * B[9];
    return dist2(B, px, py, pz, nx, ny, nz) <= r2;
}

// Integer box holding every node of a sphere (grown by `pad` nodes).
struct Box {
    int x0, y0, z0, ex, ey, ez;
};

__device__ __forceinline__ Box body_box(const double *B, int pad)
{
    Box b;
    b.x0 = (int)ceil(B[0] - B[9]) - pad;
    b.y0 = (int)ceil(B[1] - B[9]) - pad;
    b.z0 = (int)ceil(B[2] - B[9]) - pad;
    b.ex = (int)floor(B[0] + B[9]) + pad - b.x0 + 1;
    b.ey = (int)floor(B[1] + B[9]) + pad - b.y0 + 1;
    b.ez = (int)floor(B[2] + B[9]) + pad - b.z0 + 1;
    return b;
}

// Rigid-body velocity V + Omega x r at node p, r the minimum image of p - X.
__device__ __forceinline__ void sphere_velocity(const double *B, int px, int py, int pz, int nx, int ny, int nz,
                                                double &u0, double &u1, double &u2)
{
    const double r0 = min_image((double)px - B[0], nx);
    const double r1 = min_image((double)py - B[1], ny);
    const double r2 = min_image((double)pz - B[2], nz);
    u0 = B[3] + (B[7] * r2 - B[8] * r1);
    u1 = B[4] + (B[8] * r0 - B[6] * r2);
    u2 = B[5] + (B[6] * r1 - B[7] * r0);
}

}  // namespace dev
}  // namespace lbm
