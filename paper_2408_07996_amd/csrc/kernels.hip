// kernels.hip -- gfx950 kernels of the adaptive event renderer.
//
// Wavefront path tracer for one piece of a sampling round (raygen, 4-wide
// BVH closest-hit and any-hit traversal, shading with next-event
// estimation and Russian roulette, grey or RGB radiance), the per-pixel
// FP64 Welford accumulator of the mini-batch log-luminance, and the fused
// t-test / decision kernel with wave-ballot compaction of the pixels that
// stay undecided.
//
// Floating point: the whole file is compiled without FMA contraction; the
// only fused multiply-adds are the explicit ones in the (conservative) box
// test, some of them mixed-precision (FP16 plane offsets).  Path arithmetic is FP32 in the order documented next to each
// step; sin, cos and log are evaluated in FP64 (sin/cos rounded to FP32)
// and statistics are FP64.
#include <algorithm>
#include <mutex>
#include <vector>

#include <hip/hip_ext.h>
#include <hipcub/device/device_radix_sort.hpp>

#include "../../include/evrt.h"
#include "evrt_kernels.h"

namespace evrt {
namespace {

// ------------------------------------------------------------------------
// Small helpers.

__device__ __forceinline__ uint32_t fdiv(const FastDiv &f, uint32_t n)
{
    return (__umulhi(n, f.m) + n) >> f.s;
}

__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float bitsf(uint32_t x) { return __uint_as_float(x); }

// Philox4x32-10 (Salmon et al., SC'11): per round the counter becomes
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key
// advances by the two Weyl increments between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // One 32x32->64 product per multiplier (a single v_mad_u64_u32).
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                       (uint32_t)p0);
    }
    return c;
}

// Random block of (pixel, sample, frame q, vertex, block): Philox counter
// (pixel, sample, (q mod 256) << 24 | vertex << 8 | block, q >> 8).
__device__ __forceinline__ uint4 rng_block(const RenderParams &rp, uint32_t pixel, uint32_t sample,
                                           uint32_t q, uint32_t vertex, uint32_t block)
{
    return philox10(make_uint4(pixel, sample, ((q & 0xffu) << 24) | (vertex << 8) | block, q >> 8), rp.key0,
                    rp.key1);
}

// Uniform in [0, 1 - 2^-24].
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

__device__ __forceinline__ float dot3f(float ax, float ay, float az, float bx, float by, float bz)
{
    return (ax * bx + ay * by) + az * bz;
}

__device__ __forceinline__ float sel3(float4 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// Appends one element per lane with pred set; returns the lane's slot.
// One atomic per wave; must be called by every active lane of the wave.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t *counter)
{
    const unsigned long long mask = __ballot(pred);
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    const uint32_t total = (uint32_t)__popcll(mask);
    uint32_t base = 0;
    if (total) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        if ((int)__lane_id() == leader) base = atomicAdd(counter, total);
        base = __shfl(base, leader);
    }
    return base + rank;
}

// Slots in two append-only queues for a 256-thread block: one device-scope
// atomic per queue and block (not per wave), so that thousands of resident
// waves do not serialize on the two counters.  Every thread of the block
// must call it the same number of times; par alternates between calls so
// that a wave running ahead cannot overwrite counts still being read.
struct BlockAppend {
    uint32_t wc[2][2][16];  // block_append2: [parity][queue][wave] counts, up to 1024-thread blocks
    uint32_t base[2][2];
// Keys per queue of the grouped appends (16 / 32 bins with 512-thread
// shade blocks: 116.3 / 115.9 ms per sensor frame).
#ifndef EVRT_BINS
#define EVRT_BINS 32
#endif
    uint32_t bin[2][2][EVRT_BINS];  // block_append_binned: [parity][queue][bin] counts, then slots
};
static_assert(EVRT_BINS <= 64 && (EVRT_BINS & (EVRT_BINS - 1)) == 0,
              "the grouped appends scan a queue's bins within one wave");

__device__ __forceinline__ void block_append2(BlockAppend &sm, uint32_t par, bool pa, bool pb, uint32_t *ca,
                                              uint32_t *cb, uint32_t &sa, uint32_t &sb)
{
    const unsigned long long ma = __ballot(pa), mb = __ballot(pb);
    const uint32_t w = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        sm.wc[par][0][w] = (uint32_t)__popcll(ma);
        sm.wc[par][1][w] = (uint32_t)__popcll(mb);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t nw = blockDim.x >> 6;
        uint32_t ta = 0, tb = 0;
        for (uint32_t v = 0; v < nw; ++v) {
            ta += sm.wc[par][0][v];
            tb += sm.wc[par][1][v];
        }
        sm.base[par][0] = ta ? atomicAdd(ca, ta) : 0u;
        sm.base[par][1] = tb ? atomicAdd(cb, tb) : 0u;
    }
    __syncthreads();
    uint32_t oa = sm.base[par][0], ob = sm.base[par][1];
    for (uint32_t v = 0; v < w; ++v) {
        oa += sm.wc[par][0][v];
        ob += sm.wc[par][1][v];
    }
    sa = oa + __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0u));
    sb = ob + __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
}

// As block_append2, but the block's entries of each queue are laid out
// grouped by a key below EVRT_BINS (the slot order within a group is arbitrary), so
// that rays of one block with similar directions are traced by the same
// waves.  Bins of parity par must be zero on entry: clear both parities
// (followed by a barrier) before the first call; each call clears the other
// parity's bins after every thread has finished the previous call.
__device__ __forceinline__ void block_append_binned(BlockAppend &sm, uint32_t par, bool pa, uint32_t key_a,
                                                    bool pb, uint32_t key_b, uint32_t *ca, uint32_t *cb,
                                                    uint32_t &sa, uint32_t &sb)
{
    uint32_t ra = 0, rb = 0;
    if (pa) ra = atomicAdd(&sm.bin[par][0][key_a % EVRT_BINS], 1u);
    if (pb) rb = atomicAdd(&sm.bin[par][1][key_b % EVRT_BINS], 1u);
    __syncthreads();
    // Threads q * EVRT_BINS + b (the first wave, or the first two with 64
    // bins) turn the counts into slots: lane-parallel scans over each
    // queue's bins give the offsets (a serial loop in one thread cost 1.3 ms
    // per sensor frame), and each queue's first thread takes the queue's
    // slots with one atomic.
    if (threadIdx.x < 2 * EVRT_BINS) {
        const uint32_t q = threadIdx.x / EVRT_BINS, b = threadIdx.x % EVRT_BINS;
        const uint32_t n = sm.bin[par][q][b];
        uint32_t v = n;
#pragma unroll
        for (int off = 1; off < EVRT_BINS; off <<= 1) {
            const uint32_t u = (uint32_t)__shfl_up((int)v, off, EVRT_BINS);
            if (b >= (uint32_t)off) v += u;
        }
        const int first = (int)((q * EVRT_BINS) & 63u);
        const uint32_t tot = (uint32_t)__shfl((int)v, first + EVRT_BINS - 1);
        uint32_t base = 0;
        if (b == 0 && tot) base = atomicAdd(q ? cb : ca, tot);
        base = (uint32_t)__shfl((int)base, first);
        sm.bin[par][q][b] = base + v - n;
        sm.bin[par ^ 1u][q][b] = 0u;
    }
    __syncthreads();
    sa = pa ? sm.bin[par][0][key_a % EVRT_BINS] + ra : 0u;
    sb = pb ? sm.bin[par][1][key_b % EVRT_BINS] + rb : 0u;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// XCD-aware split of a queue with one region per instant.  Workgroups are
// dispatched round-robin over the 8 XCDs, so with n_split = 2 the blocks of
// XCDs 0-3 take the first instant's region and those of XCDs 4-7 the
// second's: each XCD's L2 then caches one instant's geometry.
struct Part {
    uint32_t base, n, lb, lgrid;
    uint32_t r;  // region index
};

__device__ __forceinline__ Part partition(const uint32_t *cnt2, uint32_t region, uint32_t n_split)
{
    Part p;
    uint32_t r = 0;
    if (n_split == 2) {
        const uint32_t xcd = blockIdx.x & 7u;
        r = xcd >> 2;
        p.lb = (blockIdx.x >> 3) * 4u + (xcd & 3u);
        p.lgrid = (gridDim.x >> 3) * 4u;
    } else {
        p.lb = blockIdx.x;
        p.lgrid = gridDim.x;
    }
    p.r = r;
    p.base = r * region;
    p.n = cnt2[r];
    return p;
}

// ------------------------------------------------------------------------
// Ray preparation shared by both traversal kinds.

struct TRay {
    float ix, iy, iz;       // reciprocal direction (tiny components clamped)
    float nox, noy, noz;    // -origin * reciprocal, for the fused slab test
    float okx, oky, okz;    // origin permuted into the watertight frame
    float Sx, Sy, Sz;       // shear constants
    uint32_t kperm;         // kx | ky << 2 | kz << 4
    uint32_t onx, ony, onz; // byte offsets of the near planes of a 4-wide node
};

__device__ __forceinline__ float safe_dir(float d)
{
    return fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d;
}

// Watertight ray frame (Woop, Benthin, Wald 2013): z = axis of the largest
// |d| (ties to the lower axis), x and y cyclic after it, swapped when
// d_z < 0; shear Sx = d_x / d_z, Sy = d_y / d_z, Sz = 1 / d_z.
// plane_scale: the node array's power-of-two plane scale; the reciprocal
// direction is multiplied by it (exactly) after the origin terms are formed.
__device__ __forceinline__ TRay make_tray(float ox, float oy, float oz, float dx, float dy, float dz,
                                          float plane_scale)
{
    TRay r;
    // Reciprocals for the box test only (culling, covered by the padding).
    r.ix = __builtin_amdgcn_rcpf(safe_dir(dx));
    r.iy = __builtin_amdgcn_rcpf(safe_dir(dy));
    r.iz = __builtin_amdgcn_rcpf(safe_dir(dz));
    r.nox = -(ox * r.ix);
    r.noy = -(oy * r.iy);
    r.noz = -(oz * r.iz);
#if EVRT_HALF_NODES
    r.ix *= plane_scale;
    r.iy *= plane_scale;
    r.iz *= plane_scale;
#else
    (void)plane_scale;
#endif
    // Near planes: lo planes for a positive direction component, hi planes
    // for a negative one; the far planes of an axis are the other half of
    // its pair.
#if EVRT_HALF_NODES
    r.onx = r.ix < 0.0f ? 40u : 32u;
    r.ony = r.iy < 0.0f ? 64u : 56u;
    r.onz = r.iz < 0.0f ? 88u : 80u;
#else
    r.onx = r.ix < 0.0f ? 16u : 0u;
    r.ony = r.iy < 0.0f ? 48u : 32u;
    r.onz = r.iz < 0.0f ? 80u : 64u;
#endif
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int kz = 0;
    float m = ax;
    if (ay > m) { kz = 1; m = ay; }
    if (az > m) { kz = 2; }
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    const float4 d4 = make_float4(dx, dy, dz, 0.0f);
    const float dkz = sel3(d4, kz);
    if (dkz < 0.0f) { const int tmp = kx; kx = ky; ky = tmp; }
    r.kperm = (uint32_t)kx | ((uint32_t)ky << 2) | ((uint32_t)kz << 4);
    r.Sx = sel3(d4, kx) / dkz;
    r.Sy = sel3(d4, ky) / dkz;
    r.Sz = 1.0f / dkz;
    const float4 o4 = make_float4(ox, oy, oz, 0.0f);
    r.okx = sel3(o4, kx);
    r.oky = sel3(o4, ky);
    r.okz = sel3(o4, kz);
    return r;
}

// Watertight test against (v0, v1, v2); on a hit stores t = T / det.
__device__ __forceinline__ bool tri_test(const TRay &r, float4 v0, float4 v1, float4 v2, float &t)
{
    const int kx = r.kperm & 3, ky = (r.kperm >> 2) & 3, kz = r.kperm >> 4;
    const float ax = sel3(v0, kx) - r.okx, ay = sel3(v0, ky) - r.oky, az = sel3(v0, kz) - r.okz;
    const float bx = sel3(v1, kx) - r.okx, by = sel3(v1, ky) - r.oky, bz = sel3(v1, kz) - r.okz;
    const float cx = sel3(v2, kx) - r.okx, cy = sel3(v2, ky) - r.oky, cz = sel3(v2, kz) - r.okz;
    const float Ax = ax - r.Sx * az, Ay = ay - r.Sy * az;
    const float Bx = bx - r.Sx * bz, By = by - r.Sy * bz;
    const float Cx = cx - r.Sx * cz, Cy = cy - r.Sy * cz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = (U + V) + W;
    if (det == 0.0f) return false;
    const float Az = r.Sz * az, Bz = r.Sz * bz, Cz = r.Sz * cz;
    const float T = (U * Az + V * Bz) + W * Cz;
    t = T / det;
    return true;
}

// Slab test of the four child boxes of a 4-wide node against the segment
// (tmin, tfar).  Boxes are padded on the host by more than the rounding of
// the fused products, so no triangle the exact test hits is culled.  The
// result per slot is a sort key: ~0u for a miss, else the bits of the entry
// distance (>= tmin > 0, so unsigned order is distance order) with the slot
// index in the two low bits.
__device__ __forceinline__ uint32_t slot_key(float tn, float tf, uint32_t j)
{
    return tn <= tf ? ((__float_as_uint(tn) & ~3u) | j) : ~0u;
}

__device__ __forceinline__ void box4(const TRay &r, float4 nx, float4 fx, float4 ny, float4 fy, float4 nz,
                                     float4 fz, float tmin, float tfar, uint32_t (&k)[4])
{
#define EVRT_SLOT(c, j)                                                                              \
    {                                                                                                \
        const float tn = fmaxf(fmaxf(fmaxf(__builtin_fmaf(nx.c, r.ix, r.nox), __builtin_fmaf(ny.c, r.iy, r.noy)), \
                                     __builtin_fmaf(nz.c, r.iz, r.noz)), tmin);                      \
        const float tf = fminf(fminf(fminf(__builtin_fmaf(fx.c, r.ix, r.nox), __builtin_fmaf(fy.c, r.iy, r.noy)), \
                                     __builtin_fmaf(fz.c, r.iz, r.noz)), tfar);                      \
        k[j] = slot_key(tn, tf, j);                                                                  \
    }
    EVRT_SLOT(x, 0)
    EVRT_SLOT(y, 1)
    EVRT_SLOT(z, 2)
    EVRT_SLOT(w, 3)
#undef EVRT_SLOT
}

#if EVRT_HALF_NODES
__device__ __forceinline__ float half_lo(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// The same slab test on FP16 planes stored as offsets h from the node
// origin p: with B = p inv - o inv (o the ray origin; one fused product per
// axis), the plane p + h enters as fma(h, inv, B), the FP16-to-FP32
// conversion folded into a mixed-precision FMA.  (p, h and inv carry the
// tree's power-of-two plane scale, which cancels exactly.)  near/far hold
// the four children's planes of one axis (child 2j in the low half of word
// j).  The second rounding (of B) is far inside the host's box padding;
// the offsets are rounded outward.
__device__ __forceinline__ void box4h(const TRay &r, float4 org, uint2 nx, uint2 fx, uint2 ny, uint2 fy,
                                      uint2 nz, uint2 fz, float tmin, float tfar, uint32_t (&k)[4])
{
    const float bx = __builtin_fmaf(org.x, r.ix, r.nox);
    const float by = __builtin_fmaf(org.y, r.iy, r.noy);
    const float bz = __builtin_fmaf(org.z, r.iz, r.noz);
#define EVRT_SLOT(w, H, j)                                                                           \
    {                                                                                                \
        const float tn = fmaxf(fmaxf(fmaxf(__builtin_fmaf(H(nx.w), r.ix, bx), __builtin_fmaf(H(ny.w), r.iy, by)), \
                                     __builtin_fmaf(H(nz.w), r.iz, bz)), tmin);                      \
        const float tf = fminf(fminf(fminf(__builtin_fmaf(H(fx.w), r.ix, bx), __builtin_fmaf(H(fy.w), r.iy, by)), \
                                     __builtin_fmaf(H(fz.w), r.iz, bz)), tfar);                      \
        k[j] = slot_key(tn, tf, j);                                                                  \
    }
    EVRT_SLOT(x, half_lo, 0)
    EVRT_SLOT(x, half_hi, 1)
    EVRT_SLOT(y, half_lo, 2)
    EVRT_SLOT(y, half_hi, 3)
#undef EVRT_SLOT
}

#endif

// Traversal block shape: kTB threads, a top treelet of kLdsNodes nodes per
// instant staged in LDS, and a per-lane stack whose first kStackLds entries
// live in LDS (deeper entries spill to private memory).
#ifndef EVRT_STACK_LDS
#define EVRT_STACK_LDS 16
#endif
#ifndef EVRT_LDS_NODES
#define EVRT_LDS_NODES 32
#endif
#ifndef EVRT_TRACE_WAVES
#define EVRT_TRACE_WAVES 8
#endif
constexpr int kTB = 256;
constexpr int kLdsNodes = EVRT_LDS_NODES;
constexpr int kStackLds = EVRT_STACK_LDS;
// A visit pushes at most three children, so a tree of D inner levels needs
// at most 3 D entries; the builder's depth bound keeps D <= kStackMax / 3.
constexpr int kStackMax = 96;


// Per-lane traversal state: the ray, the open segment (tmin, tmax), the
// current far bound (closest hit so far, or tmax for any-hit), the next
// reference to process and the stack depth.
struct Trav {
    TRay r;
    float tmin, tmax, tfar;
    uint32_t skip, best_p;
    int32_t ref;
    int sp;
};

// LDS-typed pointers keep LDS accesses as ds_read/ds_write (a generic
// pointer that may also point elsewhere compiles to flat accesses).
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) float lds_f32;

// The geometry one traversal reads: the node and triangle arrays of an
// instant, its root, and the first n_lds nodes staged in LDS at lds.  The
// trace kernels take one instant per block, so that these are uniform.
struct Geo {
    const float4 *nodes;
    const float4 *tris;
    const lds_f32 *lds;
    uint32_t n_lds;
    int32_t root;
    float scale;  // the node array's plane scale
};

__device__ __forceinline__ Geo make_geo(const DevScene &sc, uint32_t inst, const lds_f32 *lds)
{
    Geo g;
    g.nodes = inst ? sc.inst[1].nodes : sc.inst[0].nodes;
    g.tris = inst ? sc.inst[1].tris : sc.inst[0].tris;
    g.n_lds = inst ? sc.inst[1].n_lds : sc.inst[0].n_lds;
    g.root = inst ? sc.inst[1].root : sc.inst[0].root;
    g.scale = inst ? sc.inst[1].plane_scale : sc.inst[0].plane_scale;
    g.lds = lds;
    return g;
}

__device__ __forceinline__ void trav_begin(Trav &T, const Geo &g, float ox, float oy, float oz, float dx,
                                           float dy, float dz, float tmin, float tmax, uint32_t skip)
{
    const int32_t root = g.root;
    T.r = make_tray(ox, oy, oz, dx, dy, dz, g.scale);
    T.tmin = tmin;
    T.tmax = tmax;
    T.tfar = tmax;
    T.skip = skip;
    T.best_p = kNoPrim;
    T.ref = root;
    T.sp = 0;
}

__device__ __forceinline__ float4 lds_load4(const lds_f32 *p)
{
    return make_float4(p[0], p[1], p[2], p[3]);
}

// Stack entry sp: LDS for the first kStackLds entries, private memory
// beyond (the LDS read is always issued in bounds so that it stays a plain
// LDS access).
__device__ __forceinline__ int32_t stack_pop(int sp, const lds_u32 *lds_stack, const int32_t *spill)
{
    int32_t v = (int32_t)lds_stack[min(sp, kStackLds - 1) * kTB];
    if (sp >= kStackLds) v = spill[sp - kStackLds];
    return v;
}

__device__ __forceinline__ void stack_push(int &sp, int32_t v, lds_u32 *lds_stack, int32_t *spill)
{
    if (sp < kStackLds) lds_stack[sp * kTB] = (uint32_t)v;
    else spill[sp - kStackLds] = v;
    ++sp;
}

// Ordered descent through one 4-wide node given its children's sort keys
// and references: go to the nearest hit child and push the other hit
// children farthest first, or pop when none is hit.  Returns false when the
// stack is empty (traversal complete).
__device__ __forceinline__ bool visit_node(Trav &T, uint32_t (&k)[4], float4 refs, lds_u32 *lds_stack,
                                           int32_t *spill)
{
    int32_t c[4] = {__float_as_int(refs.x), __float_as_int(refs.y), __float_as_int(refs.z), __float_as_int(refs.w)};
    // Sorting network on (key, reference) pairs; misses sort last.
#define EVRT_CSWAP(a, b)                                   \
    {                                                      \
        const bool sw = k[b] < k[a];                       \
        const uint32_t ka = sw ? k[b] : k[a];              \
        const uint32_t kb = sw ? k[a] : k[b];              \
        const int32_t ca = sw ? c[b] : c[a];               \
        const int32_t cb = sw ? c[a] : c[b];               \
        k[a] = ka;                                         \
        k[b] = kb;                                         \
        c[a] = ca;                                         \
        c[b] = cb;                                         \
    }
    EVRT_CSWAP(0, 1)
    EVRT_CSWAP(2, 3)
    EVRT_CSWAP(0, 2)
    EVRT_CSWAP(1, 3)
    EVRT_CSWAP(1, 2)
#undef EVRT_CSWAP
    if (k[0] != ~0u) {
        T.ref = c[0];
        if (T.sp + 3 <= kStackLds) {
            // Hits are sorted first: write all three candidates, advancing
            // only past hits (a miss is overwritten by the next write or
            // left above the stack top).
            lds_stack[T.sp * kTB] = (uint32_t)c[3];
            T.sp += k[3] != ~0u;
            lds_stack[T.sp * kTB] = (uint32_t)c[2];
            T.sp += k[2] != ~0u;
            lds_stack[T.sp * kTB] = (uint32_t)c[1];
            T.sp += k[1] != ~0u;
        } else {
            if (k[3] != ~0u) stack_push(T.sp, c[3], lds_stack, spill);
            if (k[2] != ~0u) stack_push(T.sp, c[2], lds_stack, spill);
            if (k[1] != ~0u) stack_push(T.sp, c[1], lds_stack, spill);
        }
        return true;
    }
    if (T.sp == 0) return false;
    --T.sp;
    T.ref = stack_pop(T.sp, lds_stack, spill);
    return true;
}

// Row of a node array at a 32-bit byte offset (a uniform base plus one
// 32-bit offset register per load).
__device__ __forceinline__ float4 row_at(const float4 *base, uint32_t off)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

// Four words at a 32-bit byte offset that is a multiple of 8 (global
// vector loads need only 4-byte alignment).
typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ u32x4a words_at(const float4 *base, uint32_t off)
{
    return *reinterpret_cast<const u32x4a *>(reinterpret_cast<const char *>(base) + off);
}

// An empty statement that takes the reference row as an input: the row is
// then loaded with the plane rows instead of being sunk into the hit branch,
// which would add a dependent memory round trip to most visits (134.6 vs
// 137.0 ms per sensor frame).
__device__ __forceinline__ void keep_loaded(float4 refs)
{
    asm volatile("" ::"v"(refs.x), "v"(refs.y), "v"(refs.z), "v"(refs.w));
}

// Sort keys and child references of the 4-wide node at byte offset b of
// the global node array.
__device__ __forceinline__ float4 node_keys(const Trav &T, const float4 *nodes, uint32_t b, uint32_t (&k)[4])
{
#if EVRT_HALF_NODES
    // An axis's planes are stored as [lo01 lo23 hi01 hi23 lo01 lo23]; one
    // 16 B load at the ray's offset returns its near words then its far
    // words.  All five loads are issued before the statement that pins the
    // reference row, which would otherwise order the plane loads after it.
    const float4 org = row_at(nodes, b);
    const u32x4a rx = words_at(nodes, b + T.r.onx);
    const u32x4a ry = words_at(nodes, b + T.r.ony);
    const u32x4a rz = words_at(nodes, b + T.r.onz);
    const float4 refs = row_at(nodes, b + 16u);
    keep_loaded(refs);
    const uint2 nx = make_uint2(rx.x, rx.y), fx = make_uint2(rx.z, rx.w);
    const uint2 ny = make_uint2(ry.x, ry.y), fy = make_uint2(ry.z, ry.w);
    const uint2 nz = make_uint2(rz.x, rz.y), fz = make_uint2(rz.z, rz.w);
    box4h(T.r, org, nx, fx, ny, fy, nz, fz, T.tmin, T.tfar, k);
#else
    const float4 nx = row_at(nodes, b + T.r.onx), fx = row_at(nodes, b + (T.r.onx ^ 16u));
    const float4 ny = row_at(nodes, b + T.r.ony), fy = row_at(nodes, b + (T.r.ony ^ 16u));
    const float4 nz = row_at(nodes, b + T.r.onz), fz = row_at(nodes, b + (T.r.onz ^ 16u));
    const float4 refs = row_at(nodes, b + 96u);
    keep_loaded(refs);
    box4(T.r, nx, fx, ny, fy, nz, fz, T.tmin, T.tfar, k);
#endif
    return refs;
}

// The same for a node of the LDS treelet starting at p.
__device__ __forceinline__ float4 node_keys_lds(const Trav &T, const lds_f32 *p, uint32_t (&k)[4])
{
#if EVRT_HALF_NODES
    const float4 org = lds_load4(p);
    const lds_u32 *q = reinterpret_cast<const lds_u32 *>(p);
    const uint32_t ox = T.r.onx / 4, oy = T.r.ony / 4, oz = T.r.onz / 4;
    const uint2 nx = make_uint2(q[ox], q[ox + 1]), fx = make_uint2(q[ox + 2], q[ox + 3]);
    const uint2 ny = make_uint2(q[oy], q[oy + 1]), fy = make_uint2(q[oy + 2], q[oy + 3]);
    const uint2 nz = make_uint2(q[oz], q[oz + 1]), fz = make_uint2(q[oz + 2], q[oz + 3]);
    const float4 refs = lds_load4(p + 4);
    keep_loaded(refs);
    box4h(T.r, org, nx, fx, ny, fy, nz, fz, T.tmin, T.tfar, k);
#else
    const float4 nx = lds_load4(p + T.r.onx / 4), fx = lds_load4(p + (T.r.onx ^ 16u) / 4);
    const float4 ny = lds_load4(p + T.r.ony / 4), fy = lds_load4(p + (T.r.ony ^ 16u) / 4);
    const float4 nz = lds_load4(p + T.r.onz / 4), fz = lds_load4(p + (T.r.onz ^ 16u) / 4);
    const float4 refs = lds_load4(p + 24);
    keep_loaded(refs);
    box4(T.r, nx, fx, ny, fy, nz, fz, T.tmin, T.tfar, k);
#endif
    return refs;
}

// Tests the triangles of leaf `ref`: closest-hit keeps the lexicographic
// minimum (t, primitive) in T.tfar / T.best_p; ANY returns true at the
// first accepted hit.
template <bool ANY, bool COUNT>
__device__ __forceinline__ bool test_leaf(Trav &T, const Geo &g, int32_t ref, uint32_t &tests)
{
    const uint32_t packed = ~(uint32_t)ref;
    const uint32_t first = packed >> kLeafCountBits;
    const uint32_t count = (packed & (kMaxLeafTris - 1)) + 1;
    for (uint32_t k = 0; k < count; ++k) {
        const float4 *tp = g.tris + 3 * (size_t)(first + k);
        const float4 v0 = tp[0], v1 = tp[1], v2 = tp[2];
        const uint32_t prim = fbits(v0.w);
        if (COUNT) tests += prim != T.skip;
        float t;
        // The test runs before the origin-primitive check so that the
        // three vertex loads issue together.
        const bool h = tri_test(T.r, v0, v1, v2, t);
        if (!h || prim == T.skip) continue;
        if (!(t > T.tmin) || !(t < T.tmax)) continue;
        if (ANY) {
            T.best_p = prim;
            return true;
        }
        if (t < T.tfar || (t == T.tfar && prim < T.best_p)) {
            T.tfar = t;
            T.best_p = prim;
        }
    }
    return false;
}

// One outer iteration of the while-while traversal: inner nodes of the LDS
// treelet, inner nodes in global memory, then one leaf.  ANY stops at the
// first accepted hit.  Returns false when the ray is finished; the result is
// T.tfar / T.best_p.
// LDS: the top treelet is staged in LDS (else every node is read from
// global memory and the treelet loop is compiled out).
template <bool ANY, bool COUNT, bool LDS = true>
__device__ __forceinline__ bool traverse_step(Trav &T, const Geo &g, lds_u32 *lds_stack, int32_t *spill,
                                              uint32_t &visits, uint32_t &tests)
{
    const uint32_t n_lds = LDS ? g.n_lds : 0u;
    bool live = true;
    if (LDS) {
        while (live && T.ref >= 0 && (uint32_t)T.ref < n_lds) {
            const lds_f32 *p = g.lds + 32 * T.ref;
            if (COUNT) ++visits;
            uint32_t k[4];
            const float4 refs = node_keys_lds(T, p, k);
            live = visit_node(T, k, refs, lds_stack, spill);
        }
    }
    while (live && T.ref >= 0 && (!LDS || (uint32_t)T.ref >= n_lds)) {
        // 32-bit byte offsets: the host keeps node arrays below 4 GiB.
        const uint32_t b = (uint32_t)T.ref << 7;
        if (COUNT) ++visits;
        uint32_t k[4];
        const float4 refs = node_keys(T, g.nodes, b, k);
        live = visit_node(T, k, refs, lds_stack, spill);
    }
    if (!live) return false;
    // A pop in the global loop can return a treelet node: not a leaf yet.
    if (LDS && T.ref >= 0) return true;
    if (test_leaf<ANY, COUNT>(T, g, T.ref, tests)) return false;
    if (T.sp == 0) return false;
    --T.sp;
    T.ref = stack_pop(T.sp, lds_stack, spill);
    return true;
}

// Lanes still looking for their leaf below which the speculative node loop
// hands over to the leaf tests (1 / 2 / 4 / 6 / 8 / 12 / 16: 113.3 / 110.6 /
// 109.0 / 108.3 / 108.3 / 108.6 / 110.0 ms per sensor frame; 1 waits for
// every lane).
#ifndef EVRT_SPEC_LACK
#define EVRT_SPEC_LACK 8
#endif
constexpr int kSpecLack = EVRT_SPEC_LACK;

// The same step with speculation (nodes in global memory only): a lane
// that reaches a leaf sets it aside and goes on with its stack while other
// lanes of the wave still look for their leaf; the set-aside leaves are
// tested together.  T.ref == kEmptyRef marks a lane with nothing left
// after its set-aside leaf.
template <bool ANY, bool COUNT>
__device__ __forceinline__ bool traverse_step_spec(Trav &T, const Geo &g, lds_u32 *lds_stack, int32_t *spill,
                                                   uint32_t &visits, uint32_t &tests)
{
    int32_t leaf = kEmptyRef;
    for (;;) {
        if (T.ref < 0 && T.ref != kEmptyRef && leaf == kEmptyRef) {
            leaf = T.ref;
            if (T.sp == 0) {
                T.ref = kEmptyRef;
            } else {
                --T.sp;
                T.ref = stack_pop(T.sp, lds_stack, spill);
            }
        }
        const bool node = T.ref >= 0;
        // The node loop ends when no lane still looks for its leaf, or when
        // fewer than kSpecLack lanes do and some lane holds one: the wave
        // then tests the leaves it has and the lanes still looking go on in
        // the next step, instead of the wave following a few lanes' long
        // searches.  Every step visits a node or tests a leaf.
        const unsigned long long lack = __ballot(node && leaf == kEmptyRef);
        if (lack == 0ull) break;
        if (__popcll(lack) < kSpecLack && __any(leaf != kEmptyRef)) break;
        if (node) {
            const uint32_t b = (uint32_t)T.ref << 7;
            if (COUNT) ++visits;
            uint32_t k[4];
            const float4 refs = node_keys(T, g.nodes, b, k);
            if (!visit_node(T, k, refs, lds_stack, spill)) T.ref = kEmptyRef;
        }
    }
    // Lanes leave the compiled loop at different iterations; taking `leaf`
    // through an empty statement makes the test below read each lane's own
    // register instead of a lane mask formed inside the loop.
    asm volatile("" : "+v"(leaf));
    if (leaf != kEmptyRef && test_leaf<ANY, COUNT>(T, g, leaf, tests)) return false;
    return T.ref != kEmptyRef;
}

// Step used by the trace kernels: speculative unless a treelet is staged in
// LDS (123.8 vs 134.9 ms per sensor frame, identical outputs).
template <bool ANY, bool COUNT, bool LDS>
__device__ __forceinline__ bool trace_step(Trav &T, const Geo &g, lds_u32 *lds_stack, int32_t *spill,
                                           uint32_t &visits, uint32_t &tests)
{
    if (!LDS) return traverse_step_spec<ANY, COUNT>(T, g, lds_stack, spill, visits, tests);
    return traverse_step<ANY, COUNT, LDS>(T, g, lds_stack, spill, visits, tests);
}

// Full traversal of one ray.
template <bool ANY, bool COUNT>
__device__ __forceinline__ void traverse(Trav &T, const Geo &g, lds_u32 *lds_stack, uint32_t &visits,
                                         uint32_t &tests)
{
    if (T.ref == kEmptyRef) return;
    int32_t spill[kStackMax - kStackLds];
    if (g.n_lds == 0) {
        // Speculative steps, as in the trace kernels.
        while (traverse_step_spec<ANY, COUNT>(T, g, lds_stack, spill, visits, tests)) {
        }
        return;
    }
    while (traverse_step<ANY, COUNT>(T, g, lds_stack, spill, visits, tests)) {
    }
}

// Rays of one wave: the wave's share of a grid-stride walk over the queue in
// chunks of 64 (chunk k of wave w starts at (k W + w) 64 for W waves), so
// that all waves sweep the queue together and rays traced at the same time
// share BVH nodes in L2.  Idle lanes take the next rays of the sequence
// whenever at most kRefillBelow lanes of the wave are still traversing, so
// that lanes whose rays finish early do not idle until the slowest ray of
// the wave is done.  (At most 12 / 16 / 20 / 24 / 28 / 32 busy lanes:
// 114.9 / 114.0 / 113.2 / 113.1 / 113.6 / 114.4 ms per sensor frame.)
#ifndef EVRT_REFILL_BELOW
#define EVRT_REFILL_BELOW 24
#endif
constexpr uint32_t kRefillBelow = EVRT_REFILL_BELOW;

struct WaveRange {
    uint32_t next;   // position in the wave's sequence
    uint32_t w, W;   // wave index and wave count
    uint32_t n;      // queue length
    __device__ uint32_t at(uint32_t v) const { return ((v >> 6) * W + w) * 64u + (v & 63u); }
    __device__ bool done() const { return at(next) >= n; }
};

__device__ __forceinline__ WaveRange wave_range(const Part &pt)
{
    WaveRange r;
    r.next = 0;
    r.W = pt.lgrid * (kTB / 64);
    r.w = pt.lb * (kTB / 64) + (threadIdx.x >> 6);
    r.n = pt.n;
    return r;
}

// Hands the next rays of the range to the idle lanes when few lanes are
// busy; returns the lane's new item (or ~0u).  Wave-uniform control flow.
__device__ __forceinline__ uint32_t wave_refill(WaveRange &wr, bool busy)
{
    const unsigned long long bm = __ballot(busy);
    const uint32_t nb = (uint32_t)__popcll(bm);
    if (nb > kRefillBelow || wr.done()) return ~0u;
    const unsigned long long im = ~bm;
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(im >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)im, 0u));
    const uint32_t j = wr.at(wr.next + rank);
    wr.next += 64u - nb;
    return (!busy && j < wr.n) ? j : ~0u;
}

// Stages the treelets of instants [i0, i1) at s_nodes + (inst - i0) slots
// of kLdsNodes nodes; all threads of the block call it.
__device__ __forceinline__ void load_treelets(const DevScene &sc, uint32_t i0, uint32_t i1, float4 *s_nodes)
{
    for (uint32_t inst = i0; inst < i1; ++inst) {
        const uint32_t n = inst ? sc.inst[1].n_lds : sc.inst[0].n_lds;
        const float4 *src = inst ? sc.inst[1].nodes : sc.inst[0].nodes;
        for (uint32_t i = threadIdx.x; i < 8 * n; i += kTB) s_nodes[(inst - i0) * 8 * kLdsNodes + i] = src[i];
    }
    __syncthreads();
}

// ------------------------------------------------------------------------
// Kernels.

// Active-list entry i of a frame's first round: pixel i, or with a row
// order (rows[k] = image row at list row k) the same column of row
// rows[i / width].
__device__ __forceinline__ uint32_t first_entry(uint32_t i, uint32_t width, const uint32_t *rows)
{
    if (!rows) return i;
    const uint32_t k = i / width;
    return rows[k] * width + (i - k * width);
}

// Clears the per-pixel accumulators, fills the active list with every
// pixel and clears the frame counters.
__global__ void k_init_frame(uint32_t npx, uint32_t width, const uint32_t *rows, uint32_t *wf_n, double *wf_mean,
                             double *wf_m2, double *wf_ysum, uint32_t *act, uint32_t *cnt,
                             unsigned long long *stat)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * npx) {
        wf_n[i] = 0;
        wf_mean[i] = 0.0;
        wf_m2[i] = 0.0;
        wf_ysum[i] = 0.0;
    }
    if (i < npx) act[i] = first_entry(i, width, rows);
    if (i == 0) {
        cnt[kCntActive] = 0;
        cnt[kCntActive + 1] = 0;
        for (int k = 0; k < kStatCount; ++k) stat[k] = 0;
    }
}

// Camera rays of a piece: pinhole through (x + u, y + v), (u, v) from the
// vertex-0 random block or the pixel centre.
__global__ void k_raygen(Piece pc, DevScene sc, RenderParams rp, RayQueue q, uint32_t *cnt)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        cnt[kCntRay0] = pc.region;
        cnt[kCntRay0 + 1] = pc.n_inst == 2 ? pc.region : 0u;
        for (int k = 2; k < 2 * (kCntMaxDepth + 1); ++k) cnt[kCntRay0 + k] = 0;
        for (int k = 0; k < 2 * (kCntMaxDepth + 1); ++k) cnt[kCntShadow0 + k] = 0;
    }
    if (p >= pc.n_paths) return;
    const uint32_t qq = fdiv(pc.div_bp, p);
    const uint32_t s = p - qq * pc.bp;
    const uint32_t ii = fdiv(pc.div_nA, qq);
    const uint32_t a = qq - ii * pc.nA;
    const uint32_t e = pc.act[a];
    const uint32_t inst = pc.cams ? 0u : pc.inst_base + ii;
    const uint32_t pixel = pc.cams ? (e & kPixMask) : e;
    const uint32_t frame = rp.key_base + (pc.cams ? (e >> kPixBits) : inst);
    const uint32_t sample = pc.s0 + s;
    const DevCamera &cam = pc.cams ? pc.cams[e >> kPixBits] : (inst ? sc.inst[1].cam : sc.inst[0].cam);
    const uint32_t py = fdiv(sc.div_w, pixel);
    const uint32_t px = pixel - py * sc.width;
    const bool lens = sc.lens_radius > 0.0f;
    float j0 = 0.5f, j1 = 0.5f;
    uint4 rb = make_uint4(0u, 0u, 0u, 0u);
    if (rp.jitter || lens) rb = rng_block(rp, pixel, sample, frame, 0, 0);
    if (rp.jitter) {
        j0 = u01(rb.x);
        j1 = u01(rb.y);
    }
    const float fx = (float)px + j0, fy = (float)py + j1;
    const float nx = (2.0f * fx) / (float)sc.width - 1.0f;
    const float ny = 1.0f - (2.0f * fy) / (float)sc.height;
    const float ca = nx * cam.sx, cb = ny * cam.sy;
    float dx = (cam.fwd[0] + ca * cam.right[0]) + cb * cam.up[0];
    float dy = (cam.fwd[1] + ca * cam.right[1]) + cb * cam.up[1];
    float dz = (cam.fwd[2] + ca * cam.right[2]) + cb * cam.up[2];
    float ox = cam.eye[0], oy = cam.eye[1], oz = cam.eye[2];
    if (lens) {
        // Thin lens: a point of the aperture disk (radius R sqrt(u2), angle
        // 2 pi u3 from the same block) toward the pinhole ray's point on the
        // plane in focus, eye + F (f + a r + b u').
        const float rl = sc.lens_radius * sqrtf(u01(rb.z));
        const double ph = kTwoPi * (double)u01(rb.w);
        double sd, cd;
        sincos(ph, &sd, &cd);
        const float lu = rl * (float)cd, lv = rl * (float)sd;
        const float gx = cam.eye[0] + sc.focus_dist * dx;
        const float gy = cam.eye[1] + sc.focus_dist * dy;
        const float gz = cam.eye[2] + sc.focus_dist * dz;
        ox = (cam.eye[0] + lu * cam.right[0]) + lv * cam.up[0];
        oy = (cam.eye[1] + lu * cam.right[1]) + lv * cam.up[1];
        oz = (cam.eye[2] + lu * cam.right[2]) + lv * cam.up[2];
        dx = gx - ox;
        dy = gy - oy;
        dz = gz - oz;
    }
    const float len = sqrtf((dx * dx + dy * dy) + dz * dz);
    dx = dx / len; dy = dy / len; dz = dz / len;
    q.o[p] = make_float4(ox, oy, oz, 1.0f);
    q.d[p] = make_float4(dx, dy, dz, bitsf(p | (inst << 31)));
    q.skip[p] = kNoPrim;
    if (q.bgb) q.bgb[p] = make_float2(1.0f, 1.0f);
    pc.rad[a * pc.rs_a + ii * pc.rs_i + s] = 0.0f;
}

// Closest hit of the queued rays; hit[i] = (t, prim bits), prim = kNoPrim on
// a miss.  Grid-stride over the device-side queue count, one ray per lane.
// Region r of the queue holds rays of instant inst_base + r only.
template <bool COUNT, bool LDS>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(EVRT_TRACE_WAVES))) void k_trace_closest(DevScene sc, RayQueue q, const uint32_t *cnt_in,
                                                       uint32_t region, uint32_t n_split, uint32_t inst_base,
                                                       float2 *hit, int stat_kind, unsigned long long *stat)
{
    __shared__ float4 s_nodes[8 * kLdsNodes];
    __shared__ uint32_t s_stack[kStackLds * kTB];
    const Part pt = partition(cnt_in, region, n_split);
    const uint32_t inst = inst_base + pt.r;
    if (LDS) load_treelets(sc, inst, inst + 1, s_nodes);
    const Geo g = make_geo(sc, inst, (const lds_f32 *)s_nodes);
    if (pt.lb == 0 && threadIdx.x == 0 && pt.n) atomicAdd(stat + stat_kind, (unsigned long long)pt.n);
    uint32_t visits = 0, tests = 0;
    int32_t spill[kStackMax - kStackLds];
    lds_u32 *lds_stack = (lds_u32 *)s_stack + threadIdx.x;
    WaveRange wr = wave_range(pt);
    Trav T;
    uint32_t cur = 0;
    bool busy = false;
    for (;;) {
        const uint32_t j = wave_refill(wr, busy);
        if (j != ~0u) {
            cur = pt.base + j;
            const float4 o = q.o[cur], d = q.d[cur];
            trav_begin(T, g, o.x, o.y, o.z, d.x, d.y, d.z, kRayTmin, INFINITY, q.skip[cur]);
            busy = T.ref != kEmptyRef;
            if (!busy) hit[cur] = make_float2(T.tfar, bitsf(T.best_p));
        }
        if (!__any(busy)) {
            if (wr.done()) break;
            continue;
        }
        if (busy && !trace_step<false, COUNT, LDS>(T, g, lds_stack, spill, visits, tests)) {
            busy = false;
            hit[cur] = make_float2(T.tfar, bitsf(T.best_p));
        }
    }
    if (COUNT) {
        const unsigned long long v = wave_sum_u64(visits), t = wave_sum_u64(tests);
        if (__lane_id() == 0) {
            atomicAdd(stat + kStatNodes, v);
            atomicAdd(stat + kStatTris, t);
        }
    }
}

// FP64 gradient accumulators of a block (LDS, 2 n_mat entries) added to
// adj.g with one atomic per nonzero entry; all threads of the block call it.
__device__ __forceinline__ void adj_flush(const double *s_acc, const Adjoint &adj)
{
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < 2 * adj.n_mat; k += blockDim.x)
        if (s_acc[k] != 0.0) atomicAdd(&adj.g[k], s_acc[k]);
}

__device__ __forceinline__ void adj_clear(double *s_acc, const Adjoint &adj)
{
    for (uint32_t k = threadIdx.x; k < 2 * adj.n_mat; k += blockDim.x) s_acc[k] = 0.0;
}

// Adjoint term of an unoccluded area-light slot of shadow entry e.
__device__ __forceinline__ void shadow_adj(const DevScene &sc, const Adjoint &adj, uint32_t e, float c,
                                           double *s_acc)
{
    const double w = adj.sw[e];
    if (w == 0.0) return;
    const uint32_t emat = adj.semat[e];
    atomicAdd(&s_acc[adj.n_mat + emat], w * (double)c / (double)sc.mat[emat].y);
}

// Shadow entries: the n_slots rays of an entry share its origin; the
// contributions of the unoccluded slots are summed in slot order and added
// to the path radiance once.
// ADJ: the adjoint replay also adds w c / Le of every unoccluded area-light
// slot to the sampled emitter's material.
// LOG: vis_log[radiance index] receives the entry's mask of unoccluded
// slots (n_slots <= 32), which k_shadow_replay reads back.
template <bool COUNT, bool LDS, bool ADJ, bool LOG = false>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(EVRT_TRACE_WAVES))) void k_trace_shadow(DevScene sc, ShadowQueue sq, uint32_t n_slots,
                                                      const uint32_t *cnt_in, uint32_t region,
                                                      uint32_t n_split, uint32_t inst_base, float *rad,
                                                      unsigned long long *stat, Adjoint adj, uint32_t *vis_log)
{
    __shared__ float4 s_nodes[8 * kLdsNodes];
    __shared__ uint32_t s_stack[kStackLds * kTB];
    extern __shared__ double s_acc[];
    if (ADJ) {
        adj_clear(s_acc, adj);
        __syncthreads();
    }
    const Part pt = partition(cnt_in, region, n_split);
    const uint32_t inst = inst_base + pt.r;
    if (LDS) load_treelets(sc, inst, inst + 1, s_nodes);
    const Geo g = make_geo(sc, inst, (const lds_f32 *)s_nodes);
    uint32_t visits = 0, tests = 0, rays = 0;
    int32_t spill[kStackMax - kStackLds];
    lds_u32 *lds_stack = (lds_u32 *)s_stack + threadIdx.x;
    WaveRange wr = wave_range(pt);
    Trav T;
    uint32_t e = 0, slot = 0, vmask = 0;
    float sum = 0.0f, c = 0.0f;
    bool busy = false;     // an entry is in progress
    bool tracing = false;  // its slot `slot` is being traced
    for (;;) {
        const uint32_t j = wave_refill(wr, busy);
        if (j != ~0u) {
            e = pt.base + j;
            slot = 0;
            sum = 0.0f;
            if (LOG) vmask = 0;
            busy = true;
        }
        // Start the next slot with a contribution, or end the entry after
        // its last slot.
        while (busy && !tracing) {
            if (slot >= n_slots) {
                const uint32_t ri = fbits(sq.o[e].w);
                rad[ri] = rad[ri] + sum;
                if (LOG) vis_log[ri] = vmask;
                busy = false;
                break;
            }
            c = sq.c[slot * sq.cap + e];
            if (c > 0.0f) {
                const float4 o = sq.o[e];
                const float4 w = sq.dir[slot * sq.cap + e];
                const uint32_t meta = sq.meta[e];
                trav_begin(T, g, o.x, o.y, o.z, w.x, w.y, w.z, kRayTmin, w.w, meta & ~kInstBit);
                ++rays;
                tracing = T.ref != kEmptyRef;
                if (!tracing) {
                    sum = sum + c;
                    if (LOG) vmask |= 1u << slot;
                    if (ADJ && slot == 0) shadow_adj(sc, adj, e, c, s_acc);
                    ++slot;
                }
            } else {
                ++slot;
            }
        }
        if (!__any(busy)) {
            if (wr.done()) break;
            continue;
        }
        if (tracing && !trace_step<true, COUNT, LDS>(T, g, lds_stack, spill, visits, tests)) {
            tracing = false;
            if (T.best_p == kNoPrim) {
                sum = sum + c;
                if (LOG) vmask |= 1u << slot;
                if (ADJ && slot == 0) shadow_adj(sc, adj, e, c, s_acc);
            }
            ++slot;
            if (slot >= n_slots) {
                const uint32_t ri = fbits(sq.o[e].w);
                rad[ri] = rad[ri] + sum;
                if (LOG) vis_log[ri] = vmask;
                busy = false;
            }
        }
    }
    const unsigned long long rs = wave_sum_u64(rays);
    if (__lane_id() == 0 && rs) atomicAdd(stat + kStatShadow, rs);
    if (COUNT) {
        const unsigned long long v = wave_sum_u64(visits), t = wave_sum_u64(tests);
        if (__lane_id() == 0) {
            atomicAdd(stat + kStatNodesShadow, v);
            atomicAdd(stat + kStatTrisShadow, t);
        }
    }
    if (ADJ) adj_flush(s_acc, adj);
}

// Adjoint replay of the shadow entries from the visibility masks a logging
// forward pass wrote (k_trace_shadow with LOG): the same sums in slot order
// and the same adjoint terms, without tracing.
__global__ __launch_bounds__(256) void k_shadow_replay(DevScene sc, ShadowQueue sq, uint32_t n_slots,
                                                       const uint32_t *cnt_in, uint32_t region, uint32_t n_split,
                                                       float *rad, Adjoint adj, const uint32_t *vis_log)
{
    extern __shared__ double s_acc[];
    adj_clear(s_acc, adj);
    __syncthreads();
    for (uint32_t r = 0; r < n_split; ++r) {
        const uint32_t n = cnt_in[r];
        for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
            const uint32_t e = r * region + j;
            const uint32_t ri = fbits(sq.o[e].w);
            const uint32_t vm = vis_log[ri];
            float sum = 0.0f;
            for (uint32_t slot = 0; slot < n_slots; ++slot) {
                const float c = sq.c[slot * sq.cap + e];
                if (c > 0.0f && ((vm >> slot) & 1u)) {
                    sum = sum + c;
                    if (slot == 0) shadow_adj(sc, adj, e, c, s_acc);
                }
            }
            rad[ri] = rad[ri] + sum;
        }
    }
    adj_flush(s_acc, adj);
}

// Point light k seen from P with shading normal ns: contribution
// ((beta * fr) * I) * cos / r^2 and the shadow segment, or c = 0.
__device__ __forceinline__ float point_light_slot(const DevScene &sc, uint32_t k, float Px, float Py,
                                                  float Pz, float nsx, float nsy, float nsz,
                                                  float beta, float fr, float4 &dir)
{
    const float4 L = sc.plights[k];
    const float wx = L.x - Px, wy = L.y - Py, wz = L.z - Pz;
    const float r2 = dot3f(wx, wy, wz, wx, wy, wz);
    if (!(r2 > 0.0f)) return 0.0f;
    const float rl = sqrtf(r2);
    const float wix = wx / rl, wiy = wy / rl, wiz = wz / rl;
    const float cx = dot3f(nsx, nsy, nsz, wix, wiy, wiz);
    if (!(cx > 0.0f)) return 0.0f;
    dir = make_float4(wix, wiy, wiz, rl * kShadowScale);
    return (((beta * fr) * L.w) * cx) / r2;
}

// The same for RGB radiance: per channel throughput b3, BRDF fr3 and the
// light's intensity, reduced to luminance.
__device__ __forceinline__ float point_light_slot_rgb(const DevScene &sc, uint32_t k, float Px, float Py,
                                                      float Pz, float nsx, float nsy, float nsz,
                                                      float3 b3, float3 fr3, float4 &dir)
{
    const float4 L = sc.plights[k];
    const float wx = L.x - Px, wy = L.y - Py, wz = L.z - Pz;
    const float r2 = dot3f(wx, wy, wz, wx, wy, wz);
    if (!(r2 > 0.0f)) return 0.0f;
    const float rl = sqrtf(r2);
    const float wix = wx / rl, wiy = wy / rl, wiz = wz / rl;
    const float cx = dot3f(nsx, nsy, nsz, wix, wiy, wiz);
    if (!(cx > 0.0f)) return 0.0f;
    dir = make_float4(wix, wiy, wiz, rl * kShadowScale);
    const float4 I = sc.plights_rgb[k];
    return luminance((((b3.x * fr3.x) * I.x) * cx) / r2, (((b3.y * fr3.y) * I.y) * cx) / r2,
                     (((b3.z * fr3.z) * I.z) * cx) / r2);
}

// Shading of vertex `depth` for every queued ray: emission, next-event
// estimation (area emitters picked in proportion to area * Le, uniform
// point on the triangle; point lights), Russian roulette, cosine-weighted
// continuation.  Emits compacted shadow entries and extension rays.
// ADJ: the adjoint replay (the same shading, plus the gradient terms of the
// vertex: emission w term / Le, albedo w (L_fwd - L_before) / albedo, where
// L_before is the path radiance before this vertex's next-event estimate).
// Largest shade block: 512 threads.  The appends group a block's rays by
// key, and a larger block gives waves of fewer distinct keys while the
// block still spans few pixels (256 / 512 / 1024 threads: 120.0 / 116.4 /
// 118.7 ms per sensor frame).  Pieces with fewer than 64 samples per
// pixel, where a block spans many pixels, run 256-thread blocks whose
// appends keep the pixel order instead.
#ifndef EVRT_SHADE_TB
#define EVRT_SHADE_TB 512
#endif
constexpr int kShadeTB = EVRT_SHADE_TB;
// Radiance of the environment cube map in direction (dx, dy, dz): the
// face of the major axis (ties x, then y, then z), face coordinates
// (sc, tc) scaled by 1 / |major| from [-1, 1] to [0, N), truncated and
// clamped, FP32 operations in that order.
__device__ __forceinline__ float env_radiance(const DevScene &sc, float dx, float dy, float dz)
{
    const uint32_t N = sc.env_res;
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    uint32_t face;
    float ma, u, v;
    if (ax >= ay && ax >= az) {
        ma = ax;
        face = dx >= 0.0f ? 0u : 1u;
        u = dx >= 0.0f ? -dz : dz;
        v = -dy;
    } else if (ay >= az) {
        ma = ay;
        face = dy >= 0.0f ? 2u : 3u;
        u = dx;
        v = dy >= 0.0f ? dz : -dz;
    } else {
        ma = az;
        face = dz >= 0.0f ? 4u : 5u;
        u = dz >= 0.0f ? dx : -dx;
        v = -dy;
    }
    if (!(ma > 0.0f)) return 0.0f;
    const float fs = ((u / ma) + 1.0f) * 0.5f;
    const float ft = ((v / ma) + 1.0f) * 0.5f;
    const uint32_t i = min((uint32_t)(fs * (float)N), N - 1u);
    const uint32_t j = min((uint32_t)(ft * (float)N), N - 1u);
    return sc.env[((size_t)face * N + j) * N + i];
}

template <bool ADJ, bool RGB>
__global__ __launch_bounds__(kShadeTB) void k_shade(Piece pc, DevScene sc, RenderParams rp, RayQueue qin,
                                               const uint32_t *cnt_in, const float2 *hit,
                                               RayQueue qout, uint32_t *cnt_out, ShadowQueue sq,
                                               uint32_t *cnt_sh, uint32_t depth, Adjoint adj, float2 *hit_log)
{
    const Part pt = partition(cnt_in, pc.region, pc.n_inst);
    __shared__ BlockAppend s_app;
    extern __shared__ double s_acc[];
    uint32_t par = 0;
    for (uint32_t i = threadIdx.x; i < 4 * EVRT_BINS; i += blockDim.x)
        s_app.bin[i / (2 * EVRT_BINS)][(i / EVRT_BINS) & 1][i % EVRT_BINS] = 0u;
    if (ADJ) adj_clear(s_acc, adj);
    __syncthreads();
    // Block-uniform trip count: the appends synchronize the block.
    for (uint32_t j0 = pt.lb * blockDim.x; j0 < pt.n; j0 += pt.lgrid * blockDim.x, par ^= 1u) {
        const uint32_t j = j0 + threadIdx.x;
        const bool valid = j < pt.n;
        const uint32_t i = pt.base + (valid ? j : 0u);
        const float4 o = qin.o[i], d = qin.d[i];
        // RGB: the throughput per channel (red in o.w).
        float3 b3 = make_float3(0.0f, 0.0f, 0.0f), b3v = b3, fr3 = b3;
        if (RGB && valid) {
            const float2 bg = qin.bgb[i];
            b3 = make_float3(o.w, bg.x, bg.y);
        }
        // hit_log (per-vertex slice, by path id): the replay reads the hit the
        // logging forward pass wrote instead of a traced one.
        float2 h;
        if (ADJ && hit_log) h = hit_log[fbits(d.w) & ~kInstBit];
        else h = hit[i];
        if (!ADJ && hit_log && valid) hit_log[fbits(d.w) & ~kInstBit] = h;
        const uint32_t prim = valid ? fbits(h.y) : kNoPrim;
        bool want_shadow = false, want_ext = false;
        float Px = 0.0f, Py = 0.0f, Pz = 0.0f;
        float nsx = 0.0f, nsy = 0.0f, nsz = 0.0f, beta = 0.0f, fr = 0.0f, beta_v = 0.0f;
        float ndx = 0.0f, ndy = 0.0f, ndz = 0.0f;
        float c0 = 0.0f;
        float4 d0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        uint32_t pword = 0, ri = 0, inst = 0;
        double w = 0.0;          // ADJ: mini-batch weight of the path
        uint32_t emat = 0;       // ADJ: material of the sampled emitter
        uint32_t light = 0;      // the sampled emitter triangle (groups shadow entries)
        if (valid && prim == kNoPrim && sc.env_res) {
            // The ray leaves the scene: throughput times the environment's
            // radiance in its direction (the path ends here).
            const uint32_t p = fbits(d.w) & ~kInstBit;
            const uint32_t qq = fdiv(pc.div_bp, p);
            const uint32_t s = p - qq * pc.bp;
            const uint32_t ii = fdiv(pc.div_nA, qq);
            const uint32_t rm = (qq - ii * pc.nA) * pc.rs_a + ii * pc.rs_i + s;
            const float Lenv = env_radiance(sc, d.x, d.y, d.z);
            pc.rad[rm] = pc.rad[rm] + (RGB ? luminance(b3.x * Lenv, b3.y * Lenv, b3.z * Lenv) : o.w * Lenv);
        }
        if (prim != kNoPrim) {
            pword = fbits(d.w);
            inst = pword >> 31;
            const uint32_t p = pword & ~kInstBit;
            const uint32_t qq = fdiv(pc.div_bp, p);
            const uint32_t s = p - qq * pc.bp;
            const uint32_t ii = fdiv(pc.div_nA, qq);
            const uint32_t a = qq - ii * pc.nA;
            const uint32_t e = pc.act[a];
            const uint32_t pixel = pc.cams ? (e & kPixMask) : e;
            const uint32_t q = rp.key_base + (pc.cams ? (e >> kPixBits) : inst);
            const uint32_t sample = pc.s0 + s;
            ri = a * pc.rs_a + ii * pc.rs_i + s;
            beta = o.w;
            const float t = h.x;
            Px = o.x + t * d.x;
            Py = o.y + t * d.y;
            Pz = o.z + t * d.z;
            const float4 pr = inst ? sc.inst[1].prim[prim] : sc.inst[0].prim[prim];
            const float2 mt = sc.mat[fbits(pr.w)];
            // RGB: mt holds the largest albedo channel and the emission's
            // luminance, which drive the same decisions as grey values.
            const float alb = mt.x, Le = mt.y;
            float4 A3 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), E3 = A3;
            if (RGB) {
                A3 = sc.mat_rgb[2 * fbits(pr.w)];
                E3 = sc.mat_rgb[2 * fbits(pr.w) + 1];
            }
            const float cosi = dot3f(pr.x, pr.y, pr.z, d.x, d.y, d.z);
            nsx = cosi < 0.0f ? pr.x : -pr.x;
            nsy = cosi < 0.0f ? pr.y : -pr.y;
            nsz = cosi < 0.0f ? pr.z : -pr.z;
            if (ADJ) w = adj.W[((size_t)pixel * 2 + inst) * adj.m + sample / adj.mb];
            if (Le > 0.0f && cosi < 0.0f && (depth == 1 || !rp.nee || rp.mis)) {
                float term = RGB ? luminance(b3.x * E3.x, b3.y * E3.y, b3.z * E3.z) : beta * Le;
                if (depth > 1 && rp.nee) {
                    // MIS: this emitter point was reached by the cosine-sampled
                    // direction of the previous vertex, whose pdf cos / pi is
                    // the previous vertex's sample lz / pi (its random
                    // numbers, drawn again); next-event estimation would have
                    // sampled it with solid-angle pdf Le r^2 / (S cos_y).
                    // Power heuristic, as 1 / (1 + ratio^2).
                    const uint4 rq = rng_block(rp, pixel, sample, q, depth - 1, 1);
                    const float pb = sqrtf(fmaxf(0.0f, 1.0f - u01(rq.x))) * kInvPi;
                    const float S = inst ? sc.inst[1].emit_S : sc.inst[0].emit_S;
                    const float pl = (Le * (t * t)) / (S * (-cosi));
                    const float ratio = pl / pb;
                    term = term * (1.0f / (1.0f + ratio * ratio));
                }
                pc.rad[ri] = pc.rad[ri] + term;
                if (ADJ && w != 0.0) atomicAdd(&s_acc[adj.n_mat + fbits(pr.w)], w * (double)term / (double)Le);
            }
            if (ADJ && alb > 0.0f && w != 0.0) {
                const float Lf = adj.Lfwd[((size_t)pixel * 2 + inst) * adj.spp + sample];
                atomicAdd(&s_acc[fbits(pr.w)], w * ((double)Lf - (double)pc.rad[ri]) / (double)alb);
            }
            if (alb > 0.0f) {
                const uint4 r0 = rng_block(rp, pixel, sample, q, depth, 0);
                fr = alb * kInvPi;
                beta_v = beta;
                if (RGB) {
                    fr3 = make_float3(A3.x * kInvPi, A3.y * kInvPi, A3.z * kInvPi);
                    b3v = b3;
                }
                if (rp.nee) {
                    const uint32_t n_emit = inst ? sc.inst[1].n_emit : sc.inst[0].n_emit;
                    if (n_emit > 0) {
                        const float ul = u01(r0.x);
                        const float *cdf = inst ? sc.inst[1].emit_cdf : sc.inst[0].emit_cdf;
                        // first j with ul < cdf[j] (cdf is non-decreasing, last = 1)
                        uint32_t lo = 0, hi = n_emit - 1;
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (ul < cdf[mid]) hi = mid; else lo = mid + 1;
                        }
                        light = lo;
                        const float4 *E = (inst ? sc.inst[1].emit : sc.inst[0].emit) + 4 * (size_t)lo;
                        const float4 v0 = E[0], v1 = E[1], v2 = E[2], en = E[3];
                        const float su = sqrtf(u01(r0.y));
                        const float u2 = u01(r0.z);
                        const float w0 = 1.0f - su, w1 = su * (1.0f - u2), w2 = su * u2;
                        const float wx = ((w0 * v0.x + w1 * v1.x) + w2 * v2.x) - Px;
                        const float wy = ((w0 * v0.y + w1 * v1.y) + w2 * v2.y) - Py;
                        const float wz = ((w0 * v0.z + w1 * v1.z) + w2 * v2.z) - Pz;
                        const float r2 = dot3f(wx, wy, wz, wx, wy, wz);
                        if (r2 > 0.0f) {
                            const float rl = sqrtf(r2);
                            const float wix = wx / rl, wiy = wy / rl, wiz = wz / rl;
                            const float cx = dot3f(nsx, nsy, nsz, wix, wiy, wiz);
                            const float cy = -dot3f(en.x, en.y, en.z, wix, wiy, wiz);
                            if (cx > 0.0f && cy > 0.0f) {
                                const float S = inst ? sc.inst[1].emit_S : sc.inst[0].emit_S;
                                if (RGB) {
                                    // Per channel the grey estimate times
                                    // Le_j,c / Y(Le_j) (emitters are picked
                                    // by luminance power), then luminance.
                                    const float4 *P = inst ? sc.inst[1].prim : sc.inst[0].prim;
                                    const float4 Lq = sc.mat_rgb[2 * fbits(P[fbits(en.w)].w) + 1];
                                    c0 = luminance(((((b3.x * fr3.x) * (Lq.x / Lq.w)) * cx) * cy) * S / r2,
                                                   ((((b3.y * fr3.y) * (Lq.y / Lq.w)) * cx) * cy) * S / r2,
                                                   ((((b3.z * fr3.z) * (Lq.z / Lq.w)) * cx) * cy) * S / r2);
                                } else {
                                    c0 = ((((beta * fr) * cx) * cy) * S) / r2;
                                }
                                if (rp.mis && depth < rp.max_depth) {
                                    // MIS against the cosine-sampling pdf of the
                                    // same direction; the last vertex samples no
                                    // direction and keeps the full weight.
                                    const float pl = (v0.w * r2) / (S * cy);
                                    const float ratio = (cx * kInvPi) / pl;
                                    c0 = c0 * (1.0f / (1.0f + ratio * ratio));
                                }
                                d0 = make_float4(wix, wiy, wiz, rl * kShadowScale);
                                if (ADJ) {
                                    const float4 *P = inst ? sc.inst[1].prim : sc.inst[0].prim;
                                    emat = fbits(P[fbits(en.w)].w);
                                }
                            }
                        }
                    }
                    want_shadow = c0 > 0.0f;
                    for (uint32_t k = 0; k < sc.n_plights; ++k) {
                        float4 dk;
                        want_shadow |= (RGB ? point_light_slot_rgb(sc, k, Px, Py, Pz, nsx, nsy, nsz, b3, fr3, dk)
                                            : point_light_slot(sc, k, Px, Py, Pz, nsx, nsy, nsz, beta, fr, dk)) > 0.0f;
                    }
                }
                bool cont = depth < rp.max_depth;
                if (cont && depth >= rp.rr_start) {
                    // RGB: survival min(1, largest throughput channel).
                    const float qs = fminf(1.0f, RGB ? fmaxf(b3.x, fmaxf(b3.y, b3.z)) : beta);
                    if (u01(r0.w) >= qs) {
                        cont = false;
                    } else {
                        beta = beta / qs;
                        if (RGB) b3 = make_float3(b3.x / qs, b3.y / qs, b3.z / qs);
                    }
                }
                if (cont) {
                    const uint4 r1 = rng_block(rp, pixel, sample, q, depth, 1);
                    const float e0 = u01(r1.x), e1 = u01(r1.y);
                    const float rr = sqrtf(e0);
                    const double ph = kTwoPi * (double)e1;
                    double sd, cd;
                    sincos(ph, &sd, &cd);
                    const float cph = (float)cd, sph = (float)sd;
                    const float lx = rr * cph, ly = rr * sph, lz = sqrtf(fmaxf(0.0f, 1.0f - e0));
                    // Orthonormal basis around ns (Duff et al. 2017).
                    const float sg = copysignf(1.0f, nsz);
                    const float aa = -1.0f / (sg + nsz);
                    const float bb = (nsx * nsy) * aa;
                    const float tx = 1.0f + ((sg * nsx) * nsx) * aa, ty = sg * bb, tz = (-sg) * nsx;
                    const float bx = bb, by = sg + (nsy * nsy) * aa, bz = -nsy;
                    ndx = (tx * lx + bx * ly) + nsx * lz;
                    ndy = (ty * lx + by * ly) + nsy * lz;
                    ndz = (tz * lx + bz * ly) + nsz * lz;
                    beta = beta * alb;
                    if (RGB) b3 = make_float3(b3.x * A3.x, b3.y * A3.y, b3.z * A3.z);
                    want_ext = true;
                }
            }
        }
        const uint32_t r = pt.base / max(pc.region, 1u);
        uint32_t se, xe;
        // Within the block, shadow entries are grouped by the sampled emitter
        // and extension rays by direction octant, by whether y is the
        // dominant axis (rays off a floor all share the sign of y) and by
        // whether |x| >= |z|.
        const float ay = fabsf(ndy);
        const uint32_t oct = (ndx < 0.0f ? 1u : 0u) | (ndy < 0.0f ? 2u : 0u) | (ndz < 0.0f ? 4u : 0u) |
                             (ay >= fabsf(ndx) && ay >= fabsf(ndz) ? 8u : 0u) |
                             (EVRT_BINS >= 32 && fabsf(ndx) >= fabsf(ndz) ? 16u : 0u);
        // With fewer than 64 samples per pixel a block spans many pixels,
        // and the original (pixel-major) order keeps rays of one pixel
        // together instead.
        if (pc.bp >= 64)
            block_append_binned(s_app, par, want_shadow, light, want_ext, oct, cnt_sh + r, cnt_out + r, se, xe);
        else
            block_append2(s_app, par, want_shadow, want_ext, cnt_sh + r, cnt_out + r, se, xe);
        se += pt.base;
        xe += pt.base;
        if (want_shadow) {
            sq.o[se] = make_float4(Px, Py, Pz, bitsf(ri));
            sq.meta[se] = prim | (inst << 31);
            if (ADJ) {
                adj.sw[se] = w;
                adj.semat[se] = emat;
            }
            sq.c[se] = c0;
            if (c0 > 0.0f) sq.dir[se] = d0;
            for (uint32_t k = 0; k < sc.n_plights; ++k) {
                float4 dk = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                const float ck = RGB ? point_light_slot_rgb(sc, k, Px, Py, Pz, nsx, nsy, nsz, b3v, fr3, dk)
                                     : point_light_slot(sc, k, Px, Py, Pz, nsx, nsy, nsz, beta_v, fr, dk);
                sq.c[(k + 1) * sq.cap + se] = ck;
                if (ck > 0.0f) sq.dir[(k + 1) * sq.cap + se] = dk;
            }
        }
        if (want_ext) {
            qout.o[xe] = make_float4(Px, Py, Pz, RGB ? b3.x : beta);
            if (RGB) qout.bgb[xe] = make_float2(b3.y, b3.z);
            qout.d[xe] = make_float4(ndx, ndy, ndz, bitsf(pword));
            qout.skip[xe] = prim;
        }
    }
    if (ADJ) adj_flush(s_acc, adj);
}

// Pairwise mini-batch mean (FP32) of mb consecutive path radiances.
__device__ __forceinline__ float minibatch_mean(const float *v, uint32_t mb)
{
    if (mb == 1) return v[0];
    if (mb == 2) return (v[0] + v[1]) * 0.5f;
    if (mb == 4) return ((v[0] + v[1]) + (v[2] + v[3])) * 0.25f;
    return (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * 0.125f;
}

// Running (count, mean, M2) of x = ln(Y + eps) over mini-batch means Y of
// one pixel at one instant, and the sum of Y.
// With the normality pre-test also the third and fourth central-moment
// sums m3, m4 (slot pairs of m34; a slot with n = 0 starts them at 0).
struct Welford {
    uint32_t n;
    double mean, m2, ys;
    double m3, m4;
};

__device__ __forceinline__ Welford welford_load(uint32_t slot, const uint32_t *wf_n, const double *wf_mean,
                                                const double *wf_m2, const double *wf_ysum,
                                                const double *m34 = nullptr)
{
    Welford w{wf_n[slot], wf_mean[slot], wf_m2[slot], wf_ysum[slot], 0.0, 0.0};
    if (m34 && w.n > 0) {
        w.m3 = m34[2 * (size_t)slot];
        w.m4 = m34[2 * (size_t)slot + 1];
    }
    return w;
}

__device__ __forceinline__ void welford_store(const Welford &w, uint32_t slot, uint32_t *wf_n, double *wf_mean,
                                              double *wf_m2, double *wf_ysum, double *m34 = nullptr)
{
    wf_n[slot] = w.n;
    wf_mean[slot] = w.mean;
    wf_m2[slot] = w.m2;
    wf_ysum[slot] = w.ys;
    if (m34) {
        m34[2 * (size_t)slot] = w.m3;
        m34[2 * (size_t)slot + 1] = w.m4;
    }
}

// Welford steps over len consecutive path radiances, mb per mini-batch, in
// sample order.  With moments, the one-pass updates of the third and
// fourth central-moment sums (Pebay 2008), from the sums before the step.
__device__ __forceinline__ void welford_run(Welford &w, const float *src, uint32_t len, uint32_t mb,
                                            double log_eps, bool moments = false)
{
    for (uint32_t k = 0; k < len; k += mb) {
        const float Y = minibatch_mean(src + k, mb);
        const double x = log((double)Y + log_eps);
        w.n += 1;
        const double delta = x - w.mean;
        if (moments) {
            const double n = (double)w.n, dn = delta / n, dn2 = dn * dn, t1 = delta * dn * (n - 1.0);
            w.m4 = w.m4 + t1 * dn2 * (n * n - 3.0 * n + 3.0) + 6.0 * dn2 * w.m2 - 4.0 * dn * w.m3;
            w.m3 = w.m3 + t1 * dn * (n - 2.0) - 3.0 * dn * w.m2;
        }
        w.mean = w.mean + delta / (double)w.n;
        w.m2 = w.m2 + delta * (x - w.mean);
        w.ys = w.ys + (double)Y;
    }
}

// Normality pre-test of one accumulator (Jarque-Bera): JB = n/6 (g1^2 +
// g2^2 / 4) with skewness g1 and excess kurtosis g2 from the population
// central moments; rejected when its chi^2 (2 df) tail exp(-JB/2) < a.
// Samples without spread are not rejected.
__device__ __forceinline__ bool normality_rejected(const Welford &w, double a)
{
    const double n = (double)w.n;
    const double m2 = w.m2 / n, m3 = w.m3 / n, m4 = w.m4 / n;
    if (!(m2 > 0.0)) return false;
    const double g1sq = (m3 * m3) / (m2 * m2 * m2);
    const double g2 = m4 / (m2 * m2) - 3.0;
    const double jb = n / 6.0 * (g1sq + 0.25 * g2 * g2);
    return exp(-0.5 * jb) < a;
}

// Welford update for each mini-batch of the piece, in sample order; one
// thread per (pixel, instant).
__global__ void k_accumulate(Piece pc, RenderParams rp, uint32_t *wf_n, double *wf_mean,
                             double *wf_m2, double *wf_ysum)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= pc.nA * pc.n_inst) return;
    const uint32_t ii = g / pc.nA;
    const uint32_t a = g - ii * pc.nA;
    const uint32_t pixel = pc.act[a];
    const uint32_t slot = 2 * pixel + pc.inst_base + ii;
    Welford w = welford_load(slot, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    welford_run(w, pc.rad + a * pc.rs_a + ii * pc.rs_i, pc.bp, rp.minibatch, rp.log_eps, rp.wf_m34 != nullptr);
    welford_store(w, slot, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
}

// Eq. 7 with N = samples at the second instant; zero variance gives -inf,
// +inf or 0 by the sign of |gap| - C.
__device__ __forceinline__ double t_value(double mean0, double var0, double mean1, double var1,
                                          uint32_t m1, double C)
{
    const double gap = fabs(mean1 - mean0) - C;
    const double S = var0 + var1;
    if (S == 0.0) return gap < 0.0 ? -INFINITY : (gap > 0.0 ? INFINITY : 0.0);
    return gap / sqrt(S / (double)m1);
}

// ------------------------------------------------------------------------
// Student t lower tail P(T <= t) for real degrees of freedom df > 0, FP64,
// for tests whose df varies per pixel.  For t < 0 it is I_x(df/2, 1/2) / 2
// with x = df / (df + t^2) (the t distribution function as a regularized
// incomplete beta function), and I_x(a, b) is summed from its hypergeometric
// representation (DLMF 8.17(ii)):
//   I_x(a, b) = x^a (1 - x)^b / (a B(a, b)) * sum_n [(a + b)_n / (a + 1)_n] x^n,
// whose terms shrink at least by the factor x.  For x > 0.9 the complement
// I_x(a, 1/2) = 1 - I_y(1/2, a), y = 1 - x, is summed the same way in y.
// Relative error below 1e-10 for 1e-4 < p < 0.5, where the decisions fall,
// and below 1e-8 for p >= 1e-6; deeper in the tails the complement's
// cancellation leaves an absolute error below 1e-13 (there p << alpha).

// ln Gamma(a + 1/2) - ln Gamma(a): for a >= 40 the difference of Stirling's
// series (three correction terms, then a log1p form that keeps the O(1/a)
// remainder exact), so that large a does not cancel two large lgammas.
__device__ double lgamma_half_diff(double a)
{
    if (a < 40.0) return lgamma(a + 0.5) - lgamma(a);
    const double z = a + 0.5;
    const double iz = 1.0 / z, ia = 1.0 / a;
    const double iz2 = iz * iz, ia2 = ia * ia;
    double d = a * log1p(0.5 * ia) - 0.5 + 0.5 * log(a);
    d = d + (iz - ia) / 12.0;
    d = d - (iz * iz2 - ia * ia2) / 360.0;
    d = d + (iz * iz2 * iz2 - ia * ia2 * ia2) / 1260.0;
    return d;
}

__device__ double t_lower_tail(double t, double df)
{
    if (isnan(t) || !(df > 0.0)) return NAN;
    if (t == 0.0) return 0.5;
    if (isinf(t)) return t < 0.0 ? 0.0 : 1.0;
    const bool upper = t > 0.0;   // P(T <= t) = 1 - P(T <= -t)
    const double a = 0.5 * df;
    const double t2 = t * t;
    const double lx = -log1p(t2 / df);           // ln x
    const double x = exp(lx);
    const double y = t2 / (df + t2);
    const double ly = log(y);
    const double ln_beta = 0.5723649429247001 - lgamma_half_diff(a);  // ln B(a, 1/2); ln sqrt(pi)
    double tail;                                  // P(T <= -|t|)
    if (x <= 0.9) {
        double term = 1.0, sum = 1.0;
        for (int n = 0; n < 1000; ++n) {
            term = term * ((a + 0.5 + n) / (a + 1.0 + n) * x);
            sum = sum + term;
            if (term < 1e-17 * sum) break;
        }
        tail = 0.5 * exp(a * lx + 0.5 * ly - log(a) - ln_beta) * sum;
    } else if ((a + 0.5) * y > 200.0) {
        // |t| > sqrt(400 x): below 1e-80 at every df this branch can reach.
        tail = 0.0;
    } else {
        double term = 1.0, sum = 1.0;
        for (int n = 0; n < 1000; ++n) {
            term = term * ((a + 0.5 + n) / (1.5 + n) * y);
            sum = sum + term;
            if (term < 1e-17 * sum) break;
        }
        // I_y(1/2, a) = y^(1/2) x^a / ((1/2) B(a, 1/2)) * sum
        const double comp = exp(0.5 * ly + a * lx + 0.6931471805599453 - ln_beta) * sum;
        tail = 0.5 * (1.0 - comp);
    }
    return upper ? 1.0 - tail : tail;
}

// Degrees of freedom of the test on (m0, var0) and (m1, var1) mini-batch
// samples: pooled m0 + m1 - 2, or Welch-Satterthwaite for the variance
// estimate (var0 + var1) / m1 of Eq. 7, (var0 + var1)^2 / (var0^2 / (m0 - 1)
// + var1^2 / (m1 - 1)); the pooled value when both variances are zero.
__device__ __forceinline__ double test_df(uint32_t df_mode, uint32_t m0, double var0, uint32_t m1, double var1)
{
    const double pooled = (double)m0 + (double)m1 - 2.0;
    if (df_mode != EVRT_DF_WELCH) return pooled;
    const double S = var0 + var1;
    const double den = var0 * var0 / (double)(m0 - 1) + var1 * var1 / (double)(m1 - 1);
    return den > 0.0 ? S * S / den : pooled;
}

// Stopping rule at checkpoint j (Sec. 3.2): one-tailed, stop when t lies in
// the lower alpha tail (|gap| significantly below C); two-tailed, alpha / 2
// in either tail; mean-only, once |gap| <= C; fixed, never.
__device__ __forceinline__ bool stop_rule(const Decide &dc, uint32_t j, double t, double gap, uint32_t m0,
                                          double var0, uint32_t m1, double var1)
{
    if (dc.mode == EVRT_MODE_MEAN_ONLY) return fabs(gap) <= dc.C;
    if (dc.mode != EVRT_MODE_ADAPTIVE_1T && dc.mode != EVRT_MODE_ADAPTIVE_2T) return false;
    if (!dc.df_per_pixel) {
        if (dc.mode == EVRT_MODE_ADAPTIVE_1T) return t < dc.crit_lo[j];
        return t < dc.crit_lo[j] || t > dc.crit_hi[j];
    }
    const double df = test_df(dc.df_mode, m0, var0, m1, var1);
    if (dc.mode == EVRT_MODE_ADAPTIVE_1T) return t_lower_tail(t, df) < dc.alpha;
    return t_lower_tail(t, df) < 0.5 * dc.alpha || t_lower_tail(-t, df) < 0.5 * dc.alpha;
}

// Decision for one pixel at checkpoint j of the round (Eq. 7 against the
// checkpoint's critical values, or each pixel's own tail probability; at the
// last checkpoint of the schedule only the event rule of Alg. 1).  A
// finished pixel writes its outputs.
__device__ __forceinline__ bool decide_pixel(const Decide &dc, uint32_t j, bool final_ck, uint32_t pixel,
                                             const Welford &w0, const Welford &w1, const Outputs &out)
{
    const uint32_t m0 = w0.n, m1 = w1.n;
    const double var0 = m0 > 1 ? w0.m2 / (double)(m0 - 1) : 0.0;
    const double var1 = m1 > 1 ? w1.m2 / (double)(m1 - 1) : 0.0;
    const double t = t_value(w0.mean, var0, w1.mean, var1, m1, dc.C);
    const double gap = w1.mean - w0.mean;
    bool stop = !final_ck && stop_rule(dc, j, t, gap, m0, var0, m1, var1);
    // The normality pre-test gates early stops only (Sec. 5).
    if (stop && dc.normality_alpha > 0.0 &&
        (normality_rejected(w0, dc.normality_alpha) || normality_rejected(w1, dc.normality_alpha)))
        stop = false;
    const bool done = stop || final_ck;
    if (done) {
        out.polarity[pixel] = fabs(gap) > dc.C ? (gap > 0.0 ? 1 : -1) : 0;
        out.n_paths[pixel] = m1 * dc.minibatch;
        out.mean[2 * pixel] = w0.mean;
        out.mean[2 * pixel + 1] = w1.mean;
        out.var[2 * pixel] = var0;
        out.var[2 * pixel + 1] = var1;
        if (out.t_last) out.t_last[pixel] = t;
        if (out.mean_radiance) {
            out.mean_radiance[2 * pixel] = w0.ys / (double)m0;
            out.mean_radiance[2 * pixel + 1] = w1.ys / (double)m1;
        }
        if (out.flags) out.flags[pixel] = stop ? 1 : 0;
    }
    return done;
}

// Decision after a round for every active pixel; finished pixels write
// their outputs, the rest are compacted into act_out.
__global__ __launch_bounds__(256) void k_decide_compact(RenderParams rp, Decide dc, const uint32_t *act_in, uint32_t nA,
                                                        uint32_t *act_out, uint32_t *cnt,
                                                        const uint32_t *wf_n, const double *wf_mean,
                                                        const double *wf_m2, const double *wf_ysum,
                                                        Outputs out)
{
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    // The other round counter is free now: clear it for the next round.
    if (a == 0) cnt[kCntActive + (dc.cnt_slot ^ 1u)] = 0;
    if (a >= nA) return;
    const uint32_t pixel = act_in[a];
    const Welford w0 = welford_load(2 * pixel, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    const Welford w1 = welford_load(2 * pixel + 1, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    const bool done = decide_pixel(dc, dc.n_checks - 1, dc.final_round != 0, pixel, w0, w1, out);
    const uint32_t slot = wave_append(!done, cnt + kCntActive + dc.cnt_slot);
    if (!done) act_out[slot] = pixel;
}

// Statistics and decisions of a round whose piece holds the whole sample
// range of its pixels: checkpoint by checkpoint, the mini-batches up to the
// checkpoint enter the Welford state and the pixel is tested as if the round
// had ended there.  A pixel that stops ignores the samples traced past its
// checkpoint and keeps its state at the stop; the others are compacted into
// act_out.
__global__ __launch_bounds__(256) void k_accumulate_decide(Piece pc, RenderParams rp, Decide dc,
                                                           uint32_t *act_out, uint32_t *cnt, uint32_t *wf_n,
                                                           double *wf_mean, double *wf_m2, double *wf_ysum,
                                                           Outputs out)
{
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a == 0) cnt[kCntActive + (dc.cnt_slot ^ 1u)] = 0;
    if (a >= pc.nA) return;
    const uint32_t pixel = pc.act[a];
    Welford w0 = welford_load(2 * pixel, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    Welford w1 = welford_load(2 * pixel + 1, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    const bool moments = rp.wf_m34 != nullptr;
    const uint32_t mb = rp.minibatch;
    const float *src = pc.rad + a * pc.rs_a;
    const bool both = pc.n_inst == 2;
    uint32_t k = pc.s0;
    bool done = false;
    for (uint32_t j = 0; j < dc.n_checks; ++j) {
        const uint32_t end = dc.ck_end[j];
        if (both) {
            welford_run(w0, src + (k - pc.s0), end - k, mb, rp.log_eps, moments);
            welford_run(w1, src + pc.rs_i + (k - pc.s0), end - k, mb, rp.log_eps, moments);
        } else {
            welford_run(w1, src + (k - pc.s0), end - k, mb, rp.log_eps, moments);
        }
        k = end;
        const bool final_ck = dc.final_round != 0 && j + 1 == dc.n_checks;
        if (decide_pixel(dc, j, final_ck, pixel, w0, w1, out)) {
            done = true;
            break;
        }
    }
    // The state at the stop (or at the round's end) stays in memory: a
    // sequential video takes it as the pixel's next reference at an event.
    if (both) welford_store(w0, 2 * pixel, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    welford_store(w1, 2 * pixel + 1, wf_n, wf_mean, wf_m2, wf_ysum, rp.wf_m34);
    const uint32_t slot = wave_append(!done, cnt + kCntActive + dc.cnt_slot);
    if (!done) act_out[slot] = pixel;
}

// Start of a video frame: the current frame's statistics (second slot of
// every pixel) cleared and every pixel active; the reference slot is kept.
__global__ void k_video_frame_init(uint32_t npx, uint32_t width, const uint32_t *rows, uint32_t *wf_n,
                                   double *wf_mean, double *wf_m2, double *wf_ysum, uint32_t *act, uint32_t *cnt)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npx) {
        wf_n[2 * i + 1] = 0;
        wf_mean[2 * i + 1] = 0.0;
        wf_m2[2 * i + 1] = 0.0;
        wf_ysum[2 * i + 1] = 0.0;
        act[i] = first_entry(i, width, rows);
    }
    if (i == 0) {
        cnt[kCntActive] = 0;
        cnt[kCntActive + 1] = 0;
    }
}

// End of a video frame: a pixel that fired an event takes the frame's
// statistics as its reference (Algorithm 1 replaces the reference
// log-luminance at events only).
__global__ void k_video_update(uint32_t npx, const int8_t *polarity, uint32_t *wf_n, double *wf_mean,
                               double *wf_m2, double *wf_ysum, double *wf_m34)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npx || polarity[i] == 0) return;
    wf_n[2 * i] = wf_n[2 * i + 1];
    wf_mean[2 * i] = wf_mean[2 * i + 1];
    wf_m2[2 * i] = wf_m2[2 * i + 1];
    wf_ysum[2 * i] = wf_ysum[2 * i + 1];
    if (wf_m34) {
        wf_m34[4 * (size_t)i] = wf_m34[4 * (size_t)i + 2];
        wf_m34[4 * (size_t)i + 1] = wf_m34[4 * (size_t)i + 3];
    }
}

// ------------------------------------------------------------------------
// Frame batches: pairs (f, f + 1) of consecutive frames share the samples of
// their common frame.  Items are (frame, pixel) sample streams, traced
// whenever a pair that contains them is still undecided; decisions are per
// (pair, pixel).  State arrays are frame-major: index f * npx + pixel.

constexpr uint32_t kItemUnset = 0xffffffffu;
constexpr uint32_t kItemClaimed = 0xfffffffeu;

// Every frame's state cleared, every (frame, pixel) an item (round 0), every
// (pair, pixel) active with its two items.
__global__ void k_batch_init(uint32_t n_frames, uint32_t npx, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                             double *wf_ysum, uint32_t *item_idx, uint32_t *items, uint32_t *act, uint2 *pair_items,
                             uint32_t *cnt)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = n_frames * npx;
    if (i < n) {
        const uint32_t f = i / npx, px = i - f * npx;
        wf_n[i] = 0;
        wf_mean[i] = 0.0;
        wf_m2[i] = 0.0;
        wf_ysum[i] = 0.0;
        item_idx[i] = i;
        items[i] = (f << kPixBits) | px;
        if (f + 1 < n_frames) {
            act[i] = (f << kPixBits) | px;
            pair_items[i] = make_uint2(i, i + npx);
        }
    }
    if (i == 0) {
        cnt[kCntActive] = 0;
        cnt[kCntActive + 1] = 0;
        cnt[kCntItems] = 0;
    }
}

// Items of the round: both frames of every active pair, each once (the
// first pair to claim a (frame, pixel) appends it).  One thread per active
// pair; appends aggregated per block.
__global__ __launch_bounds__(256) void k_batch_items(const uint32_t *act, uint32_t nA, uint32_t npx,
                                                     uint32_t *item_idx, uint32_t *items, uint32_t *cnt)
{
    __shared__ BlockAppend s_app;
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    bool c0 = false, c1 = false;
    uint32_t e = 0, px = 0, f = 0;
    if (a < nA) {
        e = act[a];
        f = e >> kPixBits;
        px = e & kPixMask;
        c0 = atomicCAS(&item_idx[f * npx + px], kItemUnset, kItemClaimed) == kItemUnset;
        c1 = atomicCAS(&item_idx[(f + 1) * npx + px], kItemUnset, kItemClaimed) == kItemUnset;
    }
    uint32_t s0, s1;
    block_append2(s_app, 0, c0, c1, cnt + kCntItems, cnt + kCntItems, s0, s1);
    if (c0) {
        items[s0] = (f << kPixBits) | px;
        item_idx[f * npx + px] = s0;
    }
    if (c1) {
        items[s1] = ((f + 1) << kPixBits) | px;
        item_idx[(f + 1) * npx + px] = s1;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Items of a round sorted by (frame, pixel), written back in that order:
// every (frame, pixel) slot points at its new position, and frame_start
// holds the first position of each frame that has items (others keep
// 0xffffffff).
__global__ void k_batch_regroup(const uint32_t *sorted, uint32_t n_items, uint32_t npx, uint32_t *items,
                                uint32_t *item_idx, uint32_t *frame_start)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const uint32_t e = sorted[i];
    const uint32_t f = e >> kPixBits;
    items[i] = e;
    item_idx[f * npx + (e & kPixMask)] = i;
    if (i == 0 || (sorted[i - 1] >> kPixBits) != f) frame_start[f] = i;
}

// Item indices of both frames of every active pair.
__global__ void k_batch_pair_items(const uint32_t *act, uint32_t nA, uint32_t npx, const uint32_t *item_idx,
                                   uint2 *pair_items)
{
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nA) return;
    const uint32_t e = act[a];
    const uint32_t f = e >> kPixBits, px = e & kPixMask;
    pair_items[a] = make_uint2(item_idx[f * npx + px], item_idx[(f + 1) * npx + px]);
}

// Releases the round's items for the next round.
__global__ void k_batch_clear(const uint32_t *items, uint32_t n_items, uint32_t npx, uint32_t *item_idx,
                              uint32_t *cnt)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) cnt[kCntItems] = 0;
    if (i >= n_items) return;
    const uint32_t e = items[i];
    item_idx[(e >> kPixBits) * npx + (e & kPixMask)] = kItemUnset;
}

// Welford updates of the piece's items over the round's samples, with the
// state at every checkpoint of the round kept in snap (item-major, three
// doubles per checkpoint) when the round has more than one.
__global__ void k_batch_accumulate(Piece pc, RenderParams rp, Decide dc, uint32_t npx, uint32_t item_base,
                                   uint32_t *wf_n, double *wf_mean, double *wf_m2, double *wf_ysum, double *snap)
{
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= pc.nA) return;
    const uint32_t e = pc.act[a];
    const uint32_t slot = (e >> kPixBits) * npx + (e & kPixMask);
    Welford w = welford_load(slot, wf_n, wf_mean, wf_m2, wf_ysum);
    const float *src = pc.rad + a * pc.rs_a;
    if (dc.n_checks == 1) {
        welford_run(w, src, pc.bp, rp.minibatch, rp.log_eps);
    } else {
        uint32_t k = pc.s0;
        double *sn = snap + (size_t)(item_base + a) * dc.n_checks * 3;
        for (uint32_t j = 0; j < dc.n_checks; ++j) {
            const uint32_t end = dc.ck_end[j];
            welford_run(w, src + (k - pc.s0), end - k, rp.minibatch, rp.log_eps);
            k = end;
            sn[3 * j] = w.mean;
            sn[3 * j + 1] = w.m2;
            sn[3 * j + 2] = w.ys;
        }
    }
    welford_store(w, slot, wf_n, wf_mean, wf_m2, wf_ysum);
}

// Decisions of the active pairs at every checkpoint of the round, from the
// states (one checkpoint) or snapshots of their two frames; outputs at index
// pair * npx + pixel; undecided pairs compacted into act_out.
__global__ __launch_bounds__(256) void k_batch_decide(Decide dc, const uint32_t *act, uint32_t nA, uint32_t npx,
                                                      const uint2 *pair_items, const uint32_t *items,
                                                      const uint32_t *wf_n, const double *wf_mean,
                                                      const double *wf_m2, const double *wf_ysum,
                                                      const double *snap, uint32_t *act_out, uint32_t *cnt,
                                                      Outputs out)
{
    __shared__ BlockAppend s_app;
    const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a == 0) cnt[kCntActive + (dc.cnt_slot ^ 1u)] = 0;
    bool keep = false;
    uint32_t e = 0;
    if (a < nA) {
        e = act[a];
        const uint32_t f = e >> kPixBits, px = e & kPixMask;
        const uint32_t oi = f * npx + px;
        const uint2 it = pair_items[a];
        bool done = false;
        if (dc.n_checks == 1) {
            const Welford w0 = welford_load(f * npx + px, wf_n, wf_mean, wf_m2, wf_ysum);
            const Welford w1 = welford_load((f + 1) * npx + px, wf_n, wf_mean, wf_m2, wf_ysum);
            done = decide_pixel(dc, 0, dc.final_round != 0, oi, w0, w1, out);
        } else {
            const double *s0 = snap + (size_t)it.x * dc.n_checks * 3;
            const double *s1 = snap + (size_t)it.y * dc.n_checks * 3;
            for (uint32_t j = 0; j < dc.n_checks && !done; ++j) {
                const uint32_t m = dc.ck_end[j] / dc.minibatch;
                const Welford w0{m, s0[3 * j], s0[3 * j + 1], s0[3 * j + 2]};
                const Welford w1{m, s1[3 * j], s1[3 * j + 1], s1[3 * j + 2]};
                done = decide_pixel(dc, j, dc.final_round != 0 && j + 1 == dc.n_checks, oi, w0, w1, out);
            }
        }
        keep = !done;
    }
    uint32_t slot, unused;
    block_append2(s_app, 0, keep, false, cnt + kCntActive + dc.cnt_slot, cnt + kCntActive + dc.cnt_slot, slot,
                  unused);
    if (keep) act_out[slot] = e;
}

// Caller rays -> queue format for the trace hook.
__global__ void k_hook_rays(uint32_t n, const float *rays, const uint32_t *skip, RayQueue q,
                            float *tminmax, uint32_t *cnt)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) cnt[0] = n;
    if (i >= n) return;
    const float *r = rays + 8 * (size_t)i;
    q.o[i] = make_float4(r[0], r[1], r[2], 1.0f);
    q.d[i] = make_float4(r[4], r[5], r[6], bitsf(i));
    q.skip[i] = skip ? skip[i] : kNoPrim;
    tminmax[2 * i] = r[3];
    tminmax[2 * i + 1] = r[7];
}

// Trace hook: arbitrary (tmin, tmax) per ray, instant slot 0.
template <bool ANY>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(EVRT_TRACE_WAVES))) void k_hook_trace(DevScene sc, RayQueue q, const float *tminmax,
                                                    uint32_t n, float *t_out, uint32_t *p_out)
{
    __shared__ float4 s_nodes[8 * kLdsNodes];
    __shared__ uint32_t s_stack[kStackLds * kTB];
    load_treelets(sc, 0, 1, s_nodes);
    const Geo g = make_geo(sc, 0, (const lds_f32 *)s_nodes);
    uint32_t visits = 0, tests = 0;
    for (uint32_t i = blockIdx.x * kTB + threadIdx.x; i < n; i += gridDim.x * kTB) {
        const float4 o = q.o[i], d = q.d[i];
        Trav T;
        trav_begin(T, g, o.x, o.y, o.z, d.x, d.y, d.z, tminmax[2 * i], tminmax[2 * i + 1], q.skip[i]);
        traverse<ANY, false>(T, g, (lds_u32 *)s_stack + threadIdx.x, visits, tests);
        if (ANY) {
            p_out[i] = T.best_p != kNoPrim ? 1u : 0u;
        } else {
            if (t_out) t_out[i] = T.tfar;
            p_out[i] = T.best_p;
        }
    }
}

// Decision hook: Welford over caller samples, then the decision kernel's
// stopping and event rules; optionally the lower-tail probability of t.
__global__ void k_hook_decide(const double *x0, const double *x1, uint32_t n, uint32_t m, Decide dc,
                              double *t_out, uint8_t *stop_out, int8_t *pol_out, double *p_out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double mean[2], var[2];
    for (int s = 0; s < 2; ++s) {
        const double *x = (s ? x1 : x0) + (size_t)i * m;
        double mu = 0.0, m2 = 0.0;
        for (uint32_t k = 0; k < m; ++k) {
            const double delta = x[k] - mu;
            mu = mu + delta / (double)(k + 1);
            m2 = m2 + delta * (x[k] - mu);
        }
        mean[s] = mu;
        var[s] = m2 / (double)(m - 1);
    }
    const double t = t_value(mean[0], var[0], mean[1], var[1], m, dc.C);
    const double gap = mean[1] - mean[0];
    const bool stop = stop_rule(dc, 0, t, gap, m, var[0], m, var[1]);
    t_out[i] = t;
    stop_out[i] = stop ? 1 : 0;
    pol_out[i] = fabs(gap) > dc.C ? (gap > 0.0 ? 1 : -1) : 0;
    if (p_out) p_out[i] = t_lower_tail(t, test_df(dc.df_mode, m, var[0], m, var[1]));
}

// ------------------------------------------------------------------------
// Smoothed event loss and its gradient by path replay.

__device__ __forceinline__ double softplus_d(double z) { return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z)); }

__device__ __forceinline__ double sigmoid_d(double z)
{
    if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
    const double e = exp(z);
    return e / (1.0 + e);
}

// Zeroes the loss, the gradients and the replay mismatch count.
__global__ void k_diff_zero(double *loss, double *g, uint32_t n_g, uint32_t *mismatch)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_g) g[i] = 0.0;
    if (i == 0) {
        if (loss) *loss = 0.0;
        if (mismatch) *mismatch = 0;
    }
}

// Per pixel, from its stored path radiances L[pixel][instant][sample]: the
// mini-batch means Y_k, mu_i = (1/m) sum_k ln(Y_k + eps) (k ascending,
// FP64), Delta = mu_1 - mu_0, the loss term softplus((|Delta| - C) / tau)
// and the weight of every mini-batch in the gradient,
// W = +-sigmoid(z) sign(Delta) / tau / m / mb / (Y_k + eps) (+ at t1).
__global__ __launch_bounds__(256) void k_diff_stats(uint32_t npx, uint32_t spp, uint32_t mb, double log_eps,
                                                    double C, double tau, const double *upstream, const float *L,
                                                    double *W, double *loss, double *loss_px, double *delta_px)
{
    __shared__ double s_sum[256];
    const uint32_t px = blockIdx.x * blockDim.x + threadIdx.x;
    double lp = 0.0;
    if (px < npx) {
        const uint32_t m = spp / mb;
        double mu[2];
        for (uint32_t i = 0; i < 2; ++i) {
            const float *src = L + ((size_t)px * 2 + i) * spp;
            double sum = 0.0;
            for (uint32_t k = 0; k < m; ++k) sum += log((double)minibatch_mean(src + k * mb, mb) + log_eps);
            mu[i] = sum / (double)m;
        }
        const double delta = mu[1] - mu[0];
        // dL/dDelta: the smoothed loss's, or the caller's for a product
        // through Delta (then L = sum g Delta).
        double g;
        if (upstream) {
            g = upstream[px];
            lp = g * delta;
        } else {
            const double z = (fabs(delta) - C) / tau;
            lp = softplus_d(z);
            const double sgn = delta > 0.0 ? 1.0 : (delta < 0.0 ? -1.0 : 0.0);
            g = sigmoid_d(z) / tau * sgn;
        }
        if (loss_px) loss_px[px] = lp;
        if (delta_px) delta_px[px] = delta;
        for (uint32_t i = 0; i < 2; ++i) {
            const float *src = L + ((size_t)px * 2 + i) * spp;
            double *dst = W + ((size_t)px * 2 + i) * m;
            for (uint32_t k = 0; k < m; ++k)
                dst[k] = (i ? g : -g) / (double)m / (double)mb / ((double)minibatch_mean(src + k * mb, mb) + log_eps);
        }
    }
    s_sum[threadIdx.x] = lp;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss && s_sum[0] != 0.0) atomicAdd(loss, s_sum[0]);
}

// Replay check: count of path radiances of the replay that differ (bitwise)
// from the forward pass.
__global__ void k_diff_compare(uint64_t n, const float *a, const float *b, uint32_t *mismatch)
{
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        bad += __float_as_uint(a[i]) != __float_as_uint(b[i]) ? 1u : 0u;
    const unsigned long long t = wave_sum_u64(bad);
    if (__lane_id() == 0 && t) atomicAdd(mismatch, (uint32_t)t);
}

}  // namespace

// ------------------------------------------------------------------------
// Launch wrappers.

void launch_init_frame(hipStream_t s, uint32_t npx, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                       double *wf_ysum, uint32_t *act, uint32_t *cnt, unsigned long long *stat, uint32_t width,
                       const uint32_t *rows)
{
    const uint32_t n = 2 * npx;
    hipLaunchKernelGGL(k_init_frame, dim3(std::max(1u, (n + 255) / 256)), dim3(256), 0, s, npx,
                       std::max(1u, width), rows, wf_n, wf_mean, wf_m2, wf_ysum, act, cnt, stat);
}

void launch_raygen(hipStream_t s, const Piece &pc, const DevScene &sc, const RenderParams &rp,
                   const RayQueue &q, uint32_t *cnt)
{
    hipLaunchKernelGGL(k_raygen, dim3((pc.n_paths + 255) / 256), dim3(256), 0, s, pc, sc, rp, q, cnt);
}

void launch_trace_closest(hipStream_t s, uint32_t blocks, bool count, const DevScene &sc,
                          const RayQueue &q, const uint32_t *cnt_in, uint32_t region, uint32_t n_split,
                          uint32_t inst_base, float2 *hit, int stat_kind, unsigned long long *stat,
                          hipEvent_t ev_start, hipEvent_t ev_stop)
{
    // Start / stop events (when given) are written by the dispatch itself.
    const bool lds = sc.inst[0].n_lds > 0 || sc.inst[1].n_lds > 0;
    if (count && lds)
        hipExtLaunchKernelGGL((k_trace_closest<true, true>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop, 0, sc,
                              q, cnt_in, region, n_split, inst_base, hit, stat_kind, stat);
    else if (count)
        hipExtLaunchKernelGGL((k_trace_closest<true, false>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop, 0, sc,
                              q, cnt_in, region, n_split, inst_base, hit, stat_kind, stat);
    else if (lds)
        hipExtLaunchKernelGGL((k_trace_closest<false, true>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop, 0, sc,
                              q, cnt_in, region, n_split, inst_base, hit, stat_kind, stat);
    else
        hipExtLaunchKernelGGL((k_trace_closest<false, false>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop, 0,
                              sc, q, cnt_in, region, n_split, inst_base, hit, stat_kind, stat);
}

void launch_trace_shadow(hipStream_t s, uint32_t blocks, bool count, const DevScene &sc,
                         const ShadowQueue &sq, uint32_t n_slots, const uint32_t *cnt_in, uint32_t region,
                         uint32_t n_split, uint32_t inst_base, float *rad, unsigned long long *stat,
                         hipEvent_t ev_start, hipEvent_t ev_stop, const Adjoint *adj, uint32_t *vis_log)
{
    const bool lds = sc.inst[0].n_lds > 0 || sc.inst[1].n_lds > 0;
    const Adjoint a = adj ? *adj : Adjoint{};
    if (vis_log) {
        if (adj) {
            const uint32_t bl = blocks ? blocks : 1u;
            hipLaunchKernelGGL(k_shadow_replay, dim3(bl), dim3(256), 2 * adj->n_mat * sizeof(double), s, sc, sq,
                               n_slots, cnt_in, region, n_split, rad, a, (const uint32_t *)vis_log);
        } else {
            hipExtLaunchKernelGGL((k_trace_shadow<false, false, false, true>), dim3(blocks), dim3(kTB), 0, s,
                                  ev_start, ev_stop, 0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad,
                                  stat, a, vis_log);
        }
        return;
    }
    if (adj) {
        // The adjoint replay counts no work; its accumulators are dynamic LDS.
        const size_t sh = 2 * adj->n_mat * sizeof(double);
        if (lds)
            hipExtLaunchKernelGGL((k_trace_shadow<false, true, true>), dim3(blocks), dim3(kTB), sh, s, ev_start,
                                  ev_stop, 0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad, stat, a, nullptr);
        else
            hipExtLaunchKernelGGL((k_trace_shadow<false, false, true>), dim3(blocks), dim3(kTB), sh, s, ev_start,
                                  ev_stop, 0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad, stat, a, nullptr);
    } else if (count && lds)
        hipExtLaunchKernelGGL((k_trace_shadow<true, true, false>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop,
                              0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad, stat, a, nullptr);
    else if (count)
        hipExtLaunchKernelGGL((k_trace_shadow<true, false, false>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop,
                              0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad, stat, a, nullptr);
    else if (lds)
        hipExtLaunchKernelGGL((k_trace_shadow<false, true, false>), dim3(blocks), dim3(kTB), 0, s, ev_start, ev_stop,
                              0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad, stat, a, nullptr);
    else
        hipExtLaunchKernelGGL((k_trace_shadow<false, false, false>), dim3(blocks), dim3(kTB), 0, s, ev_start,
                              ev_stop, 0, sc, sq, n_slots, cnt_in, region, n_split, inst_base, rad, stat, a, nullptr);
}

void launch_shade(hipStream_t s, uint32_t blocks, const Piece &pc, const DevScene &sc,
                  const RenderParams &rp, const RayQueue &qin, const uint32_t *cnt_in,
                  const float2 *hit, const RayQueue &qout, uint32_t *cnt_out, const ShadowQueue &sq,
                  uint32_t *cnt_sh, uint32_t depth, uint32_t threads, const Adjoint *adj, float2 *hit_log)
{
    // threads: a multiple of 64 up to kShadeTB (the kernel is block-size agnostic).
    if (adj)
        hipLaunchKernelGGL((k_shade<true, false>), dim3(blocks), dim3(threads), 2 * adj->n_mat * sizeof(double), s,
                           pc, sc, rp, qin, cnt_in, hit, qout, cnt_out, sq, cnt_sh, depth, *adj, hit_log);
    else if (sc.rgb)
        hipLaunchKernelGGL((k_shade<false, true>), dim3(blocks), dim3(threads), 0, s, pc, sc, rp, qin, cnt_in, hit,
                           qout, cnt_out, sq, cnt_sh, depth, Adjoint{}, hit_log);
    else
        hipLaunchKernelGGL((k_shade<false, false>), dim3(blocks), dim3(threads), 0, s, pc, sc, rp, qin, cnt_in, hit,
                           qout, cnt_out, sq, cnt_sh, depth, Adjoint{}, hit_log);
}

void launch_accumulate(hipStream_t s, const Piece &pc, const RenderParams &rp, uint32_t *wf_n,
                       double *wf_mean, double *wf_m2, double *wf_ysum)
{
    const uint32_t n = pc.nA * pc.n_inst;
    hipLaunchKernelGGL(k_accumulate, dim3((n + 255) / 256), dim3(256), 0, s, pc, rp, wf_n, wf_mean,
                       wf_m2, wf_ysum);
}

void launch_accumulate_decide(hipStream_t s, const Piece &pc, const RenderParams &rp, const Decide &dc,
                              uint32_t *act_out, uint32_t *cnt, uint32_t *wf_n, double *wf_mean,
                              double *wf_m2, double *wf_ysum, const Outputs &out)
{
    hipLaunchKernelGGL(k_accumulate_decide, dim3((pc.nA + 255) / 256), dim3(256), 0, s, pc, rp, dc, act_out, cnt,
                       wf_n, wf_mean, wf_m2, wf_ysum, out);
}

void launch_decide_compact(hipStream_t s, const RenderParams &rp, const Decide &dc, const uint32_t *act_in,
                           uint32_t nA, uint32_t *act_out, uint32_t *cnt, const uint32_t *wf_n,
                           const double *wf_mean, const double *wf_m2, const double *wf_ysum,
                           const Outputs &out)
{
    hipLaunchKernelGGL(k_decide_compact, dim3((nA + 255) / 256), dim3(256), 0, s, rp, dc, act_in, nA,
                       act_out, cnt, wf_n, wf_mean, wf_m2, wf_ysum, out);
}

void launch_video_frame_init(hipStream_t s, uint32_t npx, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                             double *wf_ysum, uint32_t *act, uint32_t *cnt, uint32_t width, const uint32_t *rows)
{
    hipLaunchKernelGGL(k_video_frame_init, dim3(std::max(1u, (npx + 255) / 256)), dim3(256), 0, s, npx,
                       std::max(1u, width), rows, wf_n, wf_mean, wf_m2, wf_ysum, act, cnt);
}

void launch_video_update(hipStream_t s, uint32_t npx, const int8_t *polarity, uint32_t *wf_n, double *wf_mean,
                         double *wf_m2, double *wf_ysum, double *wf_m34)
{
    hipLaunchKernelGGL(k_video_update, dim3(std::max(1u, (npx + 255) / 256)), dim3(256), 0, s, npx, polarity, wf_n,
                       wf_mean, wf_m2, wf_ysum, wf_m34);
}

void launch_batch_init(hipStream_t s, uint32_t n_frames, uint32_t npx, uint32_t *wf_n, double *wf_mean,
                       double *wf_m2, double *wf_ysum, uint32_t *item_idx, uint32_t *items, uint32_t *act,
                       uint2 *pair_items, uint32_t *cnt)
{
    const uint32_t n = n_frames * npx;
    hipLaunchKernelGGL(k_batch_init, dim3(std::max(1u, (n + 255) / 256)), dim3(256), 0, s, n_frames, npx, wf_n,
                       wf_mean, wf_m2, wf_ysum, item_idx, items, act, pair_items, cnt);
}

void launch_batch_items(hipStream_t s, const uint32_t *act, uint32_t nA, uint32_t npx, uint32_t *item_idx,
                        uint32_t *items, uint32_t *cnt)
{
    hipLaunchKernelGGL(k_batch_items, dim3(std::max(1u, (nA + 255) / 256)), dim3(256), 0, s, act, nA, npx,
                       item_idx, items, cnt);
}

void launch_batch_pair_items(hipStream_t s, const uint32_t *act, uint32_t nA, uint32_t npx,
                             const uint32_t *item_idx, uint2 *pair_items)
{
    hipLaunchKernelGGL(k_batch_pair_items, dim3(std::max(1u, (nA + 255) / 256)), dim3(256), 0, s, act, nA, npx,
                       item_idx, pair_items);
}

size_t batch_sort_temp_bytes(uint32_t n_items)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr, n_items, 0, 32);
    return bytes;
}

void launch_batch_regroup(hipStream_t s, uint32_t *items, uint32_t n_items, uint32_t *sorted, void *temp,
                          size_t temp_bytes, uint32_t npx, uint32_t *item_idx, uint32_t *frame_start, uint32_t nf)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(std::max(1u, (nf + 255) / 256)), dim3(256), 0, s, frame_start, nf,
                       0xffffffffu);
    if (n_items == 0) return;
    size_t bytes = temp_bytes;
    const hipError_t e = hipcub::DeviceRadixSort::SortKeys(temp, bytes, (const uint32_t *)items, sorted, n_items, 0,
                                                           32, s);
    if (e != hipSuccess) return;  // reported by the caller's next HIP check
    hipLaunchKernelGGL(k_batch_regroup, dim3((n_items + 255) / 256), dim3(256), 0, s, sorted, n_items, npx, items,
                       item_idx, frame_start);
}

void launch_batch_clear(hipStream_t s, const uint32_t *items, uint32_t n_items, uint32_t npx, uint32_t *item_idx,
                        uint32_t *cnt)
{
    hipLaunchKernelGGL(k_batch_clear, dim3(std::max(1u, (n_items + 255) / 256)), dim3(256), 0, s, items, n_items,
                       npx, item_idx, cnt);
}

void launch_batch_accumulate(hipStream_t s, const Piece &pc, const RenderParams &rp, const Decide &dc,
                             uint32_t npx, uint32_t item_base, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                             double *wf_ysum, double *snap)
{
    hipLaunchKernelGGL(k_batch_accumulate, dim3((pc.nA + 255) / 256), dim3(256), 0, s, pc, rp, dc, npx, item_base,
                       wf_n, wf_mean, wf_m2, wf_ysum, snap);
}

void launch_batch_decide(hipStream_t s, const Decide &dc, const uint32_t *act, uint32_t nA, uint32_t npx,
                         const uint2 *pair_items, const uint32_t *items, const uint32_t *wf_n,
                         const double *wf_mean, const double *wf_m2, const double *wf_ysum, const double *snap,
                         uint32_t *act_out, uint32_t *cnt, const Outputs &out)
{
    hipLaunchKernelGGL(k_batch_decide, dim3(std::max(1u, (nA + 255) / 256)), dim3(256), 0, s, dc, act, nA, npx,
                       pair_items, items, wf_n, wf_mean, wf_m2, wf_ysum, snap, act_out, cnt, out);
}

void launch_diff_zero(hipStream_t s, double *loss, double *g, uint32_t n_g, uint32_t *mismatch)
{
    hipLaunchKernelGGL(k_diff_zero, dim3(std::max(1u, (n_g + 255) / 256)), dim3(256), 0, s, loss, g, n_g, mismatch);
}

void launch_diff_stats(hipStream_t s, uint32_t npx, uint32_t spp, uint32_t mb, double log_eps, double C,
                       double tau, const double *upstream, const float *L, double *W, double *loss,
                       double *loss_px, double *delta_px)
{
    hipLaunchKernelGGL(k_diff_stats, dim3((npx + 255) / 256), dim3(256), 0, s, npx, spp, mb, log_eps, C, tau,
                       upstream, L, W, loss, loss_px, delta_px);
}

void launch_diff_compare(hipStream_t s, uint64_t n, const float *a, const float *b, uint32_t *mismatch)
{
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
    if (blocks) hipLaunchKernelGGL(k_diff_compare, dim3((uint32_t)blocks), dim3(256), 0, s, n, a, b, mismatch);
}

void launch_hook_rays(hipStream_t s, uint32_t n, const float *rays, const uint32_t *skip,
                      const RayQueue &q, float *tminmax, uint32_t *cnt)
{
    hipLaunchKernelGGL(k_hook_rays, dim3((n + 255) / 256), dim3(256), 0, s, n, rays, skip, q, tminmax,
                       cnt);
}

void launch_hook_trace(hipStream_t s, uint32_t blocks, bool any, const DevScene &sc, const RayQueue &q,
                       const float *tminmax, uint32_t n, float *t_out, uint32_t *p_out)
{
    if (any)
        hipLaunchKernelGGL(k_hook_trace<true>, dim3(blocks), dim3(kTB), 0, s, sc, q, tminmax, n, t_out, p_out);
    else
        hipLaunchKernelGGL(k_hook_trace<false>, dim3(blocks), dim3(kTB), 0, s, sc, q, tminmax, n, t_out, p_out);
}

void launch_hook_decide(hipStream_t s, const double *x0, const double *x1, uint32_t n, uint32_t m,
                        const Decide &dc, double *t_out, uint8_t *stop_out, int8_t *pol_out, double *p_out)
{
    hipLaunchKernelGGL(k_hook_decide, dim3((n + 255) / 256), dim3(256), 0, s, x0, x1, n, m, dc, t_out,
                       stop_out, pol_out, p_out);
}

void kernel_occupancy(int *trace_blocks_per_cu, int *shade_blocks_per_cu)
{
    int a = 0, b = 0, c = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_trace_closest<false, false>, kTB, 0) != hipSuccess) a = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_trace_shadow<false, false, false>, kTB, 0) != hipSuccess) b = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_shade<false, false>, kShadeTB, 0) != hipSuccess) c = 1;
    *trace_blocks_per_cu = std::max(1, std::min(a, b));
    *shade_blocks_per_cu = std::max(1, c);
}

int shade_block_threads() { return kShadeTB; }
int traverse_block_threads() { return kTB; }
int lds_treelet_nodes() { return kLdsNodes; }
int traverse_max_depth() { return kStackMax / 3; }

}  // namespace evrt

// ------------------------------------------------------------------------
// Scratch of evrt_trace_rays_noalloc, for callers that cannot allocate: a
// file-scope device array; every GPU the library runs on holds its own copy
// until the process ends.  On the host the array's name only stands in for
// the symbol: host code resolves each device's address with
// hipGetSymbolAddress (once per device) and passes that address to kernels.
static __device__ __align__(256) unsigned char scratch[evrt::kNoAllocScratchBytes];

namespace evrt {

NoAllocScratch noalloc_layout(void *base)
{
    unsigned char *b = static_cast<unsigned char *>(base);
    const size_t n = kNoAllocRays;
    NoAllocScratch l;
    l.o = reinterpret_cast<float4 *>(b);
    l.d = reinterpret_cast<float4 *>(b + 16 * n);
    l.skip = reinterpret_cast<uint32_t *>(b + 32 * n);
    l.tminmax = reinterpret_cast<float *>(b + 36 * n);
    l.cnt = reinterpret_cast<uint32_t *>(b + 44 * n);
    return l;
}

hipError_t noalloc_scratch_address(int device, void **out)
{
    static std::mutex mu;
    static std::vector<void *> by_device;
    std::lock_guard<std::mutex> lock(mu);
    *out = nullptr;
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= by_device.size()) by_device.resize((size_t)device + 1, nullptr);
    if (!by_device[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        by_device[device] = p;
    }
    *out = by_device[device];
    return hipSuccess;
}

}  // namespace evrt
