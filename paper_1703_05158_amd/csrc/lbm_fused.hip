// The fused D3Q19 step on gfx950: boundary links, pull streaming, collision
// and store of a 256-node tile in one pass over HBM.
//
// Per tile (one workgroup, one node per thread):
//  1. Each thread loads the owner codes of its node and of its 18 pull
//     sources, and issues the pulls of its node whose source is fluid (the
//     streaming equation of Sec. 2.2) straight into the tile's LDS array of
//     populations.
//  2. Each fluid node marks the directions whose pull source is a solid node
//     (a cut link, Sec. 2.3); the links of the tile are listed in LDS and
//     spread over the workgroup's threads.  Per link: the value of the
//     population the node receives (the q < 1/2 and q >= 1/2 branches with
//     the moving-boundary term of eq. moving_boundary_velocity, walls at
//     q = 1/2), formed from the current state at the node and at the node
//     behind it, which the tile's pulls have brought into the caches; and
//     the momentum exchanged on the link (Sec. 2.3, force and torque), added
//     as 64-bit fixed point to the tile's LDS table of bodies.
//     The link's value goes into the LDS slot its pull would have filled.
//  3. Each node takes its 19 values from LDS; moments, the Smagorinsky
//     relaxation time, BGK + Guo collision and the store follow as in the
//     pull-collide kernel.
//  4. The tile's body sums go to the global fixed-point sums with one atomic
//     add per body and component; a small kernel turns them into the FP64
//     forces of the step.  Integer sums do not depend on the order of the
//     additions, so the forces are the same bit for bit for every launch,
//     tile shape and batch.
// The link arithmetic is that of the boundary-link pass (lbm_linkmath.h), so
// the populations equal, bit for bit, those of the link pass followed by the
// pull-collide kernel.
#include "lbm_collide.h"
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_linkmath.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <map>
#include <mutex>

namespace lbm {
namespace {

using namespace dev;

// LDS per workgroup is held to 23040 bytes, so that seven workgroups fit in
// a CU's 160 KB: 492 list items (on the duct 3-4.5% of the tiles hold more
// links and take a second round) and two copies of a 16-body force table
// (with 8 bodies, tiles 64 nodes long often found the table full and sent
// their sums to global memory)
constexpr int kLinkCap = 492;   // links of a tile listed at once (rounds beyond)
constexpr int kRec = 16;        // bodies of a tile with a slot in the LDS force table
constexpr int kCopies = 2;      // copies of the table's sums (by lane), so fewer lanes add to one address

struct FusedLds {
    uint32_t item[kLinkCap];          // link: node << 24 | I << 19 | (node behind fluid) << 18
    uint32_t val[kQ][kBlock];         // population i streamed to node n: val[i][n], as the stored value's
                                      // bits (16-bit storage: zero-extended)
    int key[kRec];                    // owner code of the body in a force slot, -1 free
    unsigned long long sum[kCopies][kRec][6];  // fixed-point F, T of that body
    int wtot[kBlock / 64];
};
static_assert(sizeof(FusedLds) <= 23040, "seven workgroups per CU");

// v 2^32 rounded to the nearest integer, ties to even, as a two's-complement
// 64-bit value.  While |v 2^32| < 2^51 one FP64 add of 1.5 2^52 leaves that
// integer in the low mantissa bits (to_fix_fast, for |v| < kFixFastLimit);
// larger values take the library conversion, which rounds the same way.
constexpr double kFixFastLimit = 524288.0;  // 2^19

__device__ __forceinline__ unsigned long long to_fix_fast(double v)
{
    constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
    const double t = __builtin_fma(v, kFixScale, kMagic);
    return (unsigned long long)(__double_as_longlong(t) - __double_as_longlong(kMagic));
}

__device__ __forceinline__ unsigned long long to_fix_slow(double v)
{
    return (unsigned long long)__double2ll_rn(v * kFixScale);
}

// Global fixed-point sums of owner code `key` (tile t picks the wall copy).
__device__ __forceinline__ unsigned long long *fix_slot(const FusedArgs &f, int key, int t)
{
    const int e = key < f.n_walls ? f.wall_base + key * kWallRep + (t & (kWallRep - 1)) : key - f.n_walls;
    return f.fsum + 6 * (size_t)e;
}

// Add one link's fixed-point force and torque to the tile's slot of body
// `key` (the lane's copy of the sums), or straight to the global sums when
// the table is full.  A slot is claimed once by compare-and-swap; later
// lookups read it.
__device__ __forceinline__ void table_add(const FusedArgs &f, FusedLds &lds, int key, const unsigned long long (&v)[6],
                                          int t)
{
    int s = key & (kRec - 1);
#pragma unroll 1
    for (int p = 0; p < kRec; ++p) {
        int cur = __hip_atomic_load(&lds.key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == -1) cur = atomicCAS(&lds.key[s], -1, key);
        if (cur == -1 || cur == key) {
            unsigned long long *d = lds.sum[threadIdx.x & (kCopies - 1)][s];
#pragma unroll
            for (int c = 0; c < 6; ++c) atomicAdd(d + c, v[c]);  // zeros too: no test per component
            return;
        }
        s = (s + 1) & (kRec - 1);
    }
    unsigned long long *g = fix_slot(f, key, t);
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (v[c]) atomicAdd(g + c, v[c]);
}

// Wait until this wavefront's vector memory loads are complete, loads into
// LDS included (s_waitcnt vmcnt(0); the compiler does not track those).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Workgroup barrier for LDS only: this wavefront's LDS operations complete,
// then s_barrier; loads from global memory, those into LDS included, stay in
// flight (a full barrier, or a fence on LDS, waits for them all).  The asm
// clobbers memory, so the compiler moves no memory access across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Exclusive prefix of cnt (0 <= cnt < 64) over the workgroup, its total, and
// whether any lane has flag set; through LDS (wtot: one word per wavefront)
// with an LDS-only barrier.
__device__ __forceinline__ int tile_scan(int cnt, bool flag, int *wtot, int &tot, bool &any)
{
    constexpr int kWaves = kBlock / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int pos = 0, wsum = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const unsigned long long mb = __ballot((cnt >> b) & 1);
        pos += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u)) << b;
        wsum += __popcll(mb) << b;
    }
    const bool wflag = __ballot(flag) != 0;  // on every lane (a ballot sees the active lanes only)
    if (lane == 0) wtot[wv] = wsum | (wflag ? 1 << 20 : 0);  // wsum < 2^13
    lds_barrier();
    tot = 0;
    int fl = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = wtot[w];
        if (w < wv) pos += t & 0xFFFFF;
        tot += t & 0xFFFFF;
        fl |= t;
    }
    any = (fl >> 20) & 1;
    return pos;
}

// Index offsets of a node's periodic neighbours along each axis: m = to the
// node at coordinate - 1, p = to the node at + 1.
struct NbOff {
    int xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ NbOff nb_off(int x, int y, int z, int nx, int ny, int nz)
{
    const int nxy = nx * ny;
    NbOff o;
    o.xm = x == 0 ? nx - 1 : -1;
    o.xp = x + 1 >= nx ? 1 - nx : 1;
    o.ym = y == 0 ? nxy - nx : -nx;
    o.yp = y + 1 >= ny ? nx - nxy : nx;
    o.zm = z == 0 ? nxy * (nz - 1) : -nxy;
    o.zp = z + 1 >= nz ? nxy * (1 - nz) : nxy;
    return o;
}

// Index of x - c_i, the source of the pull of population i (i compile-time).
__device__ __forceinline__ uint32_t pull_src(uint32_t idx, const NbOff &o, int i)
{
    int d = 0;
    if (CX[i] > 0) d += o.xm;
    if (CX[i] < 0) d += o.xp;
    if (CY[i] > 0) d += o.ym;
    if (CY[i] < 0) d += o.yp;
    if (CZ[i] > 0) d += o.zm;
    if (CZ[i] < 0) d += o.zp;
    return (uint32_t)((int)idx + d);
}

// Link j of the tile's list: its value into LDS, its momentum into the force
// table.  Walls are records like spheres: reference point, velocity, no
// spin, q = 1/2 and no minimum image (their arm is about the reference
// point).
template <int S, int TX, int TY, int TZ>
__device__ __forceinline__ void fused_link(const FusedArgs &f, FusedLds &lds, int x0, int y0, int z0, int j, int t)
{
    using St = Store<S>;
    using T = typename St::T;
    const StepArgs &a = f.s;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t it = lds.item[j];
    const int nl = (int)(it >> 24), I = (int)((it >> 19) & 31u), K = opp(I);
    const bool behind = (it >> 18) & 1u;
    const int x = x0 + nl % TX, y = y0 + (nl / TX) % TY, z = z0 + nl / (TX * TY);
    const uint32_t xi = (uint32_t)(x + nx * (y + ny * z));
    // owner code of the solid node p = x - c_I (periodic; a cache hit: the
    // node's own lane loaded it when it listed the link)
    const int os = *at(a.own, (uint32_t)(wrap_add(x, -dcx(I), nx) +
                                         nx * (wrap_add(y, -dcy(I), ny) + ny * wrap_add(z, -dcz(I), nz))));
    const bool sphere = os >= f.n_walls;
    const bool exact_q = sphere && !f.halfway;
    // the solid's record and the populations, in one round trip: the record
    // first, and the populations as stored values, converted only once all
    // are in flight (a conversion inside a branch would wait for its load,
    // and for everything issued before it)
    const double *B = sphere ? f.bodies + (size_t)(os - f.n_walls) * kBodyStride : f.wrec + (size_t)os * kBodyStride;
    const SphereK sk = sphere_k(B);
    const T rk = *at(src + (size_t)K * Ns, xi);
    T ra = T(0), rb = T(0);
    if (exact_q) {
        ra = *at(src + (size_t)I * Ns, xi);
        if (behind) {
            // the node behind x, x + c_I (periodic)
            const uint32_t xb = (uint32_t)(wrap_add(x, dcx(I), nx) + nx * (wrap_add(y, dcy(I), ny) + ny * wrap_add(z, dcz(I), nz)));
            rb = *at(src + (size_t)K * Ns, xb);
        }
    }
    const float fk = St::cvt(rk), fa = St::cvt(ra), fb = St::cvt(rb);
    const LinkGeo g = link_geo(sk, exact_q, sphere, a.rho0, x, y, z, nx, ny, nz, I);
    const float vr = St::round(link_value(g.q, fk, fa, fb, behind, g.mw));
    lds.val[I][nl] = St::to_bits(vr);  // a slot no pull is loaded into
    double acc[6];
    const double mom = link_momentum(fk, vr, I, a.rho0);
    link_force_terms(mom, I, g, acc);
    unsigned long long v[6];
    // F = -mom c_I: its fixed-point components are -c M with M = fix(mom)
    // (the rounding is odd-symmetric).  One range test for the four
    // conversions (to_fix's two ways, taken together).
    const int cI[3] = {dcx(I), dcy(I), dcz(I)};
    unsigned long long M;
    const double big =
        fmax(fmax(__builtin_fabs(mom), __builtin_fabs(acc[3])), fmax(__builtin_fabs(acc[4]), __builtin_fabs(acc[5])));
    if (big < kFixFastLimit) {
        M = to_fix_fast(mom);
#pragma unroll
        for (int c = 3; c < 6; ++c) v[c] = to_fix_fast(acc[c]);
    } else {
        M = to_fix_slow(mom);
#pragma unroll
        for (int c = 3; c < 6; ++c) v[c] = to_fix_slow(acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = cI[c] > 0 ? 0ull - M : (cI[c] < 0 ? M : 0ull);
    table_add(f, lds, os, v, t);
}

// Tile t of the lattice of f.  Every thread of the workgroup calls it (it
// holds barriers); lds may be reused by the next call.
template <int S, int TX, int TY, int TZ>
__device__ __forceinline__ void fused_tile(const FusedArgs &f, int t, FusedLds &lds)
{
    static_assert(TX * TY * TZ == kBlock, "tile must hold one workgroup");
    using St = Store<S>;
    using T = typename St::T;
    const StepArgs &a = f.s;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    const int tid = threadIdx.x;
    const int r = t / a.ntx;
    const int x0 = (t - r * a.ntx) * TX, y0 = (r % a.nty) * TY, z0 = (r / a.nty) * TZ;
    const int x = x0 + tid % TX, y = y0 + (tid / TX) % TY, z = z0 + tid / (TX * TY);
    const bool in = x < nx && y < ny && z < nz;
    const uint32_t idx = in ? (uint32_t)(x + nx * (y + ny * z)) : 0u;
    const NbOff no = nb_off(x, y, z, nx, ny, nz);
    auto src_idx = [&](int i) { return pull_src(idx, no, i); };

    // 1. owner codes of the node and of its 18 pull sources (loaded before
    //    anything else, so that waiting for them waits for nothing later)
    const uint16_t o = in ? *at(a.own, idx) : uint16_t(0);
    uint16_t on[kQ];
    if (in) {
#pragma unroll
        for (int i = 1; i < kQ; ++i) on[i] = *at(a.own, src_idx(i));
    }
    const bool fluid = in && o >= kVacated;
    lds_barrier();  // the previous tile's readers of lds are done
    // The owner codes are waited for before anything else is loaded: the
    // compiler does not count loads into LDS, so a later wait for an owner
    // code would wait for all of them.
    wait_vmem();
    uint32_t solid = 0;  // pull sources owned by a solid
    if (fluid) {
#pragma unroll
        for (int i = 1; i < kQ; ++i)
            if (on[i] < kVacated) solid |= 1u << i;
        // the node's pulls from fluid sources go straight from HBM into
        // lds.val (one word per lane, 16-bit values zero-extended), in
        // flight while the tile's links are listed and formed; the slot of
        // a cut link is left to the link's value
        constexpr int kBytes = S == 0 ? 4 : 2;  // an int: the builtin takes a 32-bit size
        const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);  // the wavefront's LDS row offset
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            if (!((solid >> i) & 1u))
                __builtin_amdgcn_global_load_lds(at(src + (size_t)i * Ns, i ? src_idx(i) : idx),
                                                 (__attribute__((address_space(3))) void *)&lds.val[i][wbase],
                                                 kBytes, 0, 0);
    }
    // cut links: not the inflow plane's directions from the removed domain
    uint32_t m = solid;
    if (z == a.zieb_z) {
#pragma unroll
        for (int i = 1; i < kQ; ++i)
            if (CZ[i] == 1) m &= ~(1u << i);
    }
    for (int k = tid; k < kRec; k += kBlock) lds.key[k] = -1;
    for (int k = tid; k < kCopies * kRec * 6; k += kBlock) (&lds.sum[0][0][0])[k] = 0ull;
    int tot;
    bool any_fluid;
    const int pos = tile_scan(__popc(m), fluid, lds.wtot, tot, any_fluid);  // its barrier also publishes the table's reset
    if (!any_fluid) return;

    // 2. the tile's links, listed and spread over the workgroup, in rounds
    //    of kLinkCap.  An item is node << 24 | I << 19 | (the node behind x
    //    is fluid) << 18; each lane walks only its own cut directions (a
    //    wavefront's walk is as long as its lanes' largest count, not 18).
    //    A link's value goes into its node's slot of lds.val, which no pull
    //    is loaded into, so the pulls stay in flight.
    // bit i: the pull source of opp(i), x + c_i, is fluid (opp pairs i, i + 9)
    const uint32_t nsolid = ~solid;
    const uint32_t behind_bits = ((nsolid >> 9) & 0x3FEu) | ((nsolid << 9) & 0x7FC00u);
    auto list = [&](int base) {  // the items with list index in [base, base + kLinkCap)
        uint32_t mm = m;
        int k = pos - base;
        while (mm) {
            const int i = __builtin_ctz(mm);
            mm &= mm - 1u;
            if (k >= 0 && k < kLinkCap)
                lds.item[k] = ((uint32_t)tid << 24) | ((uint32_t)i << 19) | (((behind_bits >> i) & 1u) << 18);
            ++k;
        }
    };
    list(0);
    for (int base = 0; base < tot; base += kLinkCap) {
        if (base) {
            lds_barrier();  // the previous round's list is processed
            list(base);
        }
        lds_barrier();  // the list is written (an LDS-only barrier: the pulls stay in flight)
        const int n = min(kLinkCap, tot - base);
        for (int j = tid; j < n; j += kBlock) fused_link<S, TX, TY, TZ>(f, lds, x0, y0, z0, j, t);
    }
    if (tot > 0) {
        __syncthreads();  // the link values and the tile's body sums are complete
        // 4. the tile's body sums, the copies added up
        if (tid < kRec) {
            const int key = lds.key[tid];
            if (key >= 0) {
                unsigned long long *gs = fix_slot(f, key, t);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    unsigned long long v = 0ull;
#pragma unroll
                    for (int q = 0; q < kCopies; ++q) v += lds.sum[q][tid][c];
                    if (v) atomicAdd(gs + c, v);
                }
            }
        }
    }

    // 3. pull, collide and store (whole wavefronts; none with no fluid lane)
    if (!in || __ballot(fluid) == 0) return;
    float g[kQ];
    wait_vmem();  // this wavefront's pulls have landed in lds.val (the link values are there since the barrier)
    if (!fluid) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) g[i] = 0.0f;
    } else {
#pragma unroll
        for (int i = 0; i < kQ; ++i) g[i] = St::from_bits(lds.val[i][tid]);
    }
    if (fluid && z == a.zieb_z) zieb_plane<S>(a, src, idx, g);
    collide_store<S>(a, g, fluid, idx, dst);
}

// Force entry i of a step (spheres, then walls) from its fixed-point sums,
// which are cleared.
__device__ __forceinline__ void finish_value(const FinishArgs &fa, int i)
{
    const int ns = 6 * fa.nb;
    unsigned long long sum;
    if (i < ns) {
        sum = fa.fsum[i];
        fa.fsum[i] = 0ull;
    } else {
        const int w = (i - ns) / 6, c = (i - ns) % 6;
        unsigned long long *p = fa.fsum + 6 * ((size_t)fa.wall_base + (size_t)w * kWallRep) + c;
        sum = 0ull;
        for (int r = 0; r < kWallRep; ++r) {
            sum += p[6 * r];
            p[6 * r] = 0ull;
        }
    }
    const double v = (double)(long long)sum * (1.0 / kFixScale);
    fa.out[i] = v;
    if (fa.out2) fa.out2[i] = v;
}

// Seven waves per SIMD: the LDS of a workgroup allows seven per CU, and the
// compiler then keeps the kernel within 72 VGPRs without spilling.
template <int S, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_fused(FusedArgs f)
{
    __shared__ FusedLds lds;
    // the previous step's forces, if nobody has read them yet (their sums
    // are in the other buffer)
    if (f.fin.fsum)
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < 6 * (f.fin.nb + f.fin.n_walls); i += gridDim.x * kBlock)
            finish_value(f.fin, i);
    fused_tile<S, TX, TY, TZ>(f, xcd_remap(blockIdx.x, gridDim.x), lds);
}

__global__ __launch_bounds__(kBlock) void k_finish(FinishArgs fa)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < 6 * (fa.nb + fa.n_walls)) finish_value(fa, i);
}

__global__ __launch_bounds__(kBlock) void k_zero_fix(unsigned long long *p, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Persistent fused step over the tiles of many lattices, all with the
// batch's tile shape.  Member m owns the global tiles [tile_begin[m],
// tile_begin[m + 1]); XCD k (workgroups k, k + 8, ...) takes its share of
// the global tile range (runs of neighbouring tiles, by xcd_item) from its
// own queue, so that each XCD works on neighbouring tiles of the same
// members while every XCD draws from all of them.  Six waves per SIMD: its
// tile loop needs more registers than seven would leave.
template <int S, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_batch_fused(BatchStepArgs b)
{
    __shared__ FusedLds lds;
    __shared__ int next[2];  // the workgroup's tile of this iteration and of the next, in turn
    const int xcd = blockIdx.x & 7;
    int *q = b.queue + xcd * kQueueStride;  // the XCD's tiles in turn, by xcd_item
    if (threadIdx.x == 0) next[0] = atomicAdd(q, 1);
    lds_barrier();
    // the member of the previous tile is kept: a workgroup's next tile is
    // usually in the same member
    int mb = 0, me = 0;
    FusedArgs f{};
    for (int k = 0;; ++k) {
        const int gt = xcd_item(xcd, __builtin_amdgcn_readfirstlane(next[k & 1]));
        if (gt >= b.total_tiles) break;  // the XCD's later items lie beyond too
        // the next tile is taken now, its atomic in flight during this one
        int pre = 0;
        if (threadIdx.x == 0) pre = atomicAdd(q, 1);
        if (gt < mb || gt >= me) {
            int m = 0, top = b.n;  // largest m with tile_begin[m] <= gt
            while (top - m > 1) {
                const int mid = (m + top) >> 1;
                if (b.members[mid].tile_begin <= gt) m = mid;
                else top = mid;
            }
            const BatchMember &bm = b.members[m];
            mb = bm.tile_begin;
            me = m + 1 < b.n ? b.members[m + 1].tile_begin : b.total_tiles;
            FusedArgs t = bm.f;
            const int c = b.cur[m];
            t.s.src = bm.pop[c];
            t.s.dst = bm.pop[c ^ 1];
            f = uniform(t);
        }
        fused_tile<S, TX, TY, TZ>(f, gt - mb, lds);
        if (threadIdx.x == 0) next[(k + 1) & 1] = pre;
        lds_barrier();
    }
}

// Forces of every member of a batch: one thread per force entry.
__global__ __launch_bounds__(kBlock) void k_batch_finish(BatchStepArgs b)
{
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= b.total_forces) return;
    int m = 0, top = b.n;  // largest m with force_begin[m] <= g
    while (top - m > 1) {
        const int mid = (m + top) >> 1;
        if (b.members[mid].force_begin <= g) m = mid;
        else top = mid;
    }
    finish_value(b.members[m].fin, g - b.members[m].force_begin);
}

__global__ __launch_bounds__(kBlock) void k_batch_flip(int *cur, int n, int *queue)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) cur[i] ^= 1;
    if (i < kQueueInts) queue[i] = 0;  // the tile queues of the next step
}

template <int S>
hipError_t launch_fused_s(const FusedArgs &f, hipStream_t s, hipEvent_t start, hipEvent_t stop)
{
    const dim3 grid(f.s.n_tiles), block(kBlock);
    void (*k)(FusedArgs) = nullptr;
    switch (f.s.tile) {
    case kTile64x2x2: k = k_fused<S, 64, 2, 2>; break;
    case kTile32x4x2: k = k_fused<S, 32, 4, 2>; break;
    case kTile32x2x4: k = k_fused<S, 32, 2, 4>; break;
    case kTile16x8x2: k = k_fused<S, 16, 8, 2>; break;
    default: return hipErrorInvalidValue;
    }
    if (start || stop)
        hipExtLaunchKernelGGL(k, grid, block, 0, s, start, stop, 0, f);
    else
        hipLaunchKernelGGL(k, grid, block, 0, s, f);
    return hipGetLastError();
}

template <int S>
const void *batch_kernel_s(int shape)
{
    switch (shape) {
    case kTile64x2x2: return (const void *)k_batch_fused<S, 64, 2, 2>;
    case kTile32x4x2: return (const void *)k_batch_fused<S, 32, 4, 2>;
    case kTile32x2x4: return (const void *)k_batch_fused<S, 32, 2, 4>;
    case kTile16x8x2: return (const void *)k_batch_fused<S, 16, 8, 2>;
    default: return nullptr;
    }
}

const void *batch_kernel(int storage, int shape)
{
    switch (storage) {
    case 0: return batch_kernel_s<0>(shape);
    case 1: return batch_kernel_s<1>(shape);
    case 2: return batch_kernel_s<2>(shape);
    default: return nullptr;
    }
}

inline int nblk(long n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_fused(int storage, const FusedArgs &f, hipStream_t s, hipEvent_t start, hipEvent_t stop)
{
    switch (storage) {
    case 0: return launch_fused_s<0>(f, s, start, stop);
    case 1: return launch_fused_s<1>(f, s, start, stop);
    case 2: return launch_fused_s<2>(f, s, start, stop);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finish(const FinishArgs &fa, hipStream_t s)
{
    const int n = 6 * (fa.nb + fa.n_walls);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3(nblk(n)), dim3(kBlock), 0, s, fa);
    return hipGetLastError();
}

hipError_t launch_zero_fix(unsigned long long *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_fix, dim3(nblk(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

// The device array behind lbm_step_noalloc's force sums.  Host code takes
// its address per device from static_fix_scratch and never uses the name.
static __device__ __align__(256) unsigned long long scratch[2 * kStaticFixHalf];

hipError_t static_fix_scratch(unsigned long long **out)
{
    static std::mutex mu;
    static std::map<int, unsigned long long *> addr;  // device -> address of scratch there
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, static_cast<unsigned long long *>(p)).first;
    }
    *out = it->second;
    return hipSuccess;
}

int batch_step_blocks_per_cu(int storage, int shape)
{
    const void *k = batch_kernel(storage, shape);
    int n = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kBlock, 0) != hipSuccess || n < 1) return 1;
    return n;
}

hipError_t launch_batch_step(int storage, int shape, const BatchStepArgs &b, int grid, hipStream_t s)
{
    if (b.total_tiles <= 0) return hipSuccess;
    const void *k = batch_kernel(storage, shape);
    if (!k) return hipErrorInvalidValue;
    BatchStepArgs arg = b;
    void *args[] = {&arg};
    return hipLaunchKernel(k, dim3(grid), dim3(kBlock), args, 0, s);
}

hipError_t launch_batch_finish(const BatchStepArgs &b, hipStream_t s)
{
    if (b.total_forces <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_finish, dim3(nblk(b.total_forces)), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_flip(int *cur, int n, int *queue, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_flip, dim3(nblk(std::max(n, kQueueInts))), dim3(kBlock), 0, s, cur, n, queue);
    return hipGetLastError();
}

}  // namespace lbm
