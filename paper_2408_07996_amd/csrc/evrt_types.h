// evrt_types.h -- plain data exchanged between the host scheduler and the
// gfx950 kernels of the adaptive event renderer.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace evrt {

constexpr uint32_t kNoPrim = 0xffffffffu;
constexpr float kRayTmin = 1e-4f;        // self-intersection offset (scene units)
constexpr float kShadowScale = 0.9999f;  // shadow segment ends short of the light
// 4-wide node format: FP16 child planes relative to a per-node origin (1),
// or FP32 planes (0).
#ifndef EVRT_HALF_NODES
#define EVRT_HALF_NODES 1
#endif

constexpr uint16_t kHalfPosInf = 0x7c00u, kHalfNegInf = 0xfc00u;

// Luminance of linear RGB with the Rec. 709 primaries (ITU-R BT.709), FP32
// operations in this order (built without contraction).
__host__ __device__ inline float luminance(float r, float g, float b)
{
    return (0.2126f * r + 0.7152f * g) + 0.0722f * b;
}
constexpr float kInvPi = 0.318309886183790671538f;
constexpr double kTwoPi = 6.283185307179586476925;
constexpr uint32_t kInstBit = 0x80000000u;  // instant flag in queue path words

// 4-wide BVH node: 128 bytes = eight float4, child slot j in component j:
//   n[0] = lo.x, n[1] = hi.x, n[2] = lo.y, n[3] = hi.y, n[4] = lo.z,
//   n[5] = hi.z, n[6] = child references (int bits), n[7] = 0.
// A reference >= 0 is an inner node, < 0 a leaf whose complement packs
// (first_triangle << 3) | (count - 1).  Unused slots hold the box
// (+inf, -inf), which no ray with finite components enters, and
// kEmptySlotRef, a leaf inside every non-empty triangle array.
constexpr int kLeafCountBits = 3;
constexpr uint32_t kMaxLeafTris = 1u << kLeafCountBits;
// Root of a scene without geometry: never decoded.  With fewer than 2^28
// triangles no leaf has this reference (it would end past 2^28).
constexpr int32_t kEmptyRef = INT32_MIN;
constexpr int32_t kEmptySlotRef = -1;  // the leaf {triangle 0}

// Unsigned division by a runtime constant for n < 2^31 (round-up method):
// q = (umulhi(n, m) + n) >> s.
struct FastDiv {
    uint32_t d, m, s;
};

struct DevCamera {
    float eye[3], fwd[3], right[3], up[3];
    float sx, sy;
};

// Geometry of the scene at one instant, device pointers.
struct DevInstant {
    const float4 *nodes;     // 8 per 4-wide inner node
    const float4 *tris;      // 3 per triangle in leaf order: (v0, prim bits), (v1, 0), (v2, 0)
    const float4 *prim;      // per primitive: (unit normal xyz, material bits)
    const float *emit_cdf;   // per emitter
    const float4 *emit;      // 4 per emitter: (v0, Le), v1, v2, (unit normal xyz, prim bits)
    int32_t root;            // root reference (kEmptyRef: no geometry)
    uint32_t n_nodes, n_lds, n_emit;
    float emit_S;            // sum over emitters of area * Le
    float plane_scale;       // power of two: node origins and FP16 plane offsets are stored divided by it
    DevCamera cam;
};

struct DevScene {
    DevInstant inst[2];
    const float2 *mat;       // (albedo, emission); RGB: (largest albedo channel, luminance of the emission)
    const float4 *plights;   // (position xyz, intensity)
    // RGB radiance (rgb = 1): per material (albedo rgb, 0), (emission rgb,
    // its luminance); per point light (intensity rgb, 0).
    const float4 *mat_rgb;
    const float4 *plights_rgb;
    uint32_t rgb;
    const float *env;        // cube map [6][env_res][env_res] (env_res 0: none)
    uint32_t n_plights;
    uint32_t env_res;
    uint32_t width, height;
    float lens_radius, focus_dist;  // thin lens (radius 0: pinhole)
    FastDiv div_w;
};

struct RenderParams {
    uint32_t key0, key1;     // Philox key
    uint32_t max_depth, rr_start;
    uint32_t nee, jitter;
    uint32_t minibatch;
    uint32_t n_slots;        // shadow rays per shade vertex: 1 + point lights
    uint32_t key_base;       // frame index of instant slot 0 in the keys
    uint32_t mis;            // 1: light samples and BSDF-sampled emitter hits
                             // weighted by the power heuristic
    double log_eps;
    // Third and fourth central-moment sums (2 per accumulator slot) for the
    // normality pre-test; null when it is off.
    double *wf_m34;
};

// A piece of a round: samples [s0, s0 + bp) of nA pixels (the active list)
// at n_inst instants starting at inst_base.  Piece-local path id
// p = (ii * nA + a) * bp + s; its radiance goes to rad[a*rs_a + ii*rs_i + s].
// Queues are split into n_inst regions of `region` slots, one per instant
// (the camera ray of path p sits at slot p).
struct Piece {
    const uint32_t *act;
    uint32_t nA, bp, n_inst, inst_base, s0;
    uint32_t n_paths, region;
    FastDiv div_bp, div_nA;
    float *rad;
    uint32_t rs_a, rs_i;
    // Frame batches: act entries are (frame << kPixBits) | pixel, the camera
    // of frame f is cams[f], geometry is slot 0 and the random-number frame
    // is key_base + f.  Null for single pairs.
    const DevCamera *cams;
};

constexpr uint32_t kPixBits = 21;                      // pixels per frame < 2^21
constexpr uint32_t kPixMask = (1u << kPixBits) - 1u;
constexpr uint32_t kMaxBatchFrames = 1u << (32 - kPixBits);

// Ray queue (SoA of float4): o = (origin xyz, throughput beta),
// d = (direction xyz, path word = p | instant << 31), skip = origin primitive;
// with RGB radiance beta is the red channel and bgb the green and blue ones
// (null otherwise).
struct RayQueue {
    float4 *o;
    float4 *d;
    uint32_t *skip;
    float2 *bgb;
};

// Shadow queue: one entry per shaded vertex with at least one shadow ray;
// n_slots rays share the origin.  o = (P xyz, radiance index bits),
// meta = skip primitive | instant << 31; slot k of entry e lives at
// [k * cap + e]: dir = (wi xyz, tmax), c = contribution (0: slot unused).
struct ShadowQueue {
    float4 *o;
    uint32_t *meta;
    float4 *dir;
    float *c;
    uint32_t cap;
};

// Device counters (uint64): rays by kind and optional work counts.
enum StatIndex : int {
    kStatCamera = 0, kStatExtension = 1, kStatShadow = 2,
    kStatNodes = 3, kStatTris = 4,          // closest-hit traversal
    kStatNodesShadow = 5, kStatTrisShadow = 6,  // any-hit traversal
    kStatCount = 8
};

}  // namespace evrt
