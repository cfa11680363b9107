// scene.cpp -- host construction of the scene at an instant: FP64
// keyframe interpolation of instances and camera, FP32 world triangles,
// per-primitive normals, the emitter table for next-event estimation, and
// a binned-SAH binary BVH collapsed into a 4-wide BVH whose top treelet is
// laid out first for LDS staging.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <future>
#include <numeric>

#include "evrt_host.h"

namespace evrt {

// Interpolation of keyed values: first key before the first key time, last
// key after the last, else v_k + w (v_{k+1} - v_k), w = (t - t_k) /
// (t_{k+1} - t_k), entry by entry in FP64.
static void keyed(const std::vector<double> &kt, const std::vector<double> &kv, size_t width,
                  double t, double *out)
{
    const size_t nk = kt.size();
    if (nk == 1 || t <= kt[0]) {
        std::memcpy(out, kv.data(), sizeof(double) * width);
        return;
    }
    if (t >= kt[nk - 1]) {
        std::memcpy(out, kv.data() + (nk - 1) * width, sizeof(double) * width);
        return;
    }
    size_t k = 0;
    while (!(t < kt[k + 1])) ++k;
    const double w = (t - kt[k]) / (kt[k + 1] - kt[k]);
    const double *a = kv.data() + k * width;
    const double *b = a + width;
    for (size_t e = 0; e < width; ++e) out[e] = a[e] + w * (b[e] - a[e]);
}

static inline uint32_t f2u(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return u;
}

static inline float u2f(uint32_t u)
{
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

void build_world(const SceneDesc &sd, double t, HostInstant &h)
{
    size_t nt = 0;
    for (const auto &in : sd.instances) nt += sd.meshes[in.mesh].mat.size();
    h.tri.assign(9 * nt, 0.0f);
    h.prim.assign(nt, make_float4(0, 0, 0, 0));
    h.area.assign(nt, 0.0f);
    size_t p = 0;
    for (const auto &in : sd.instances) {
        const MeshDesc &m = sd.meshes[in.mesh];
        double M[12];
        keyed(in.kt, in.kx, 12, t, M);
        for (size_t tr = 0; tr < m.mat.size(); ++tr, ++p) {
            float *v = &h.tri[9 * p];
            for (int c = 0; c < 3; ++c) {
                const float *src = &m.xyz[3 * (size_t)m.idx[3 * tr + c]];
                const double x = src[0], y = src[1], z = src[2];
                for (int r = 0; r < 3; ++r) {
                    const double *row = M + 4 * r;
                    v[3 * c + r] = (float)(((row[0] * x + row[1] * y) + row[2] * z) + row[3]);
                }
            }
            // Unit geometric normal and area, FP32: cross(v1 - v0, v2 - v0).
            const float e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
            const float e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
            const float gx = e1y * e2z - e1z * e2y;
            const float gy = e1z * e2x - e1x * e2z;
            const float gz = e1x * e2y - e1y * e2x;
            const float len = std::sqrt((gx * gx + gy * gy) + gz * gz);
            float4 pr;
            if (len == 0.0f) pr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            else pr = make_float4(gx / len, gy / len, gz / len, 0.0f);
            pr.w = u2f(m.mat[tr]);
            h.prim[p] = pr;
            h.area[p] = 0.5f * len;
        }
    }

    build_emitters(sd, h);
    camera_at(sd, t, h.cam);
}

void build_emitters(const SceneDesc &sd, HostInstant &h)
{
    // Emitters in primitive order: w_j = A_j * Le_j (FP32), prefix sums and
    // their total S in FP64, cdf_j = (float)(prefix_j / S), last entry 1.
    const size_t nt = h.prim.size();
    h.emit_prim.clear();
    h.emit_cdf.clear();
    std::vector<double> pref;
    double S = 0.0;
    for (size_t q = 0; q < nt; ++q) {
        const float le = sd.emission[f2u(h.prim[q].w)];
        if (le > 0.0f) {
            const float w = h.area[q] * le;
            S += (double)w;
            pref.push_back(S);
            h.emit_prim.push_back((uint32_t)q);
        }
    }
    for (double v : pref) h.emit_cdf.push_back((float)(v / S));
    if (!h.emit_cdf.empty()) h.emit_cdf.back() = 1.0f;
    h.emit_S = (float)S;
}

bool instances_static(const SceneDesc &sd, const double *times, uint32_t n)
{
    for (const auto &in : sd.instances) {
        double M0[12], M[12];
        keyed(in.kt, in.kx, 12, times[0], M0);
        for (uint32_t k = 1; k < n; ++k) {
            keyed(in.kt, in.kx, 12, times[k], M);
            if (std::memcmp(M0, M, sizeof(M)) != 0) return false;
        }
    }
    return true;
}

bool scene_static(const SceneDesc &sd)
{
    for (const auto &in : sd.instances)
        for (size_t k = 1; k < in.kt.size(); ++k)
            if (std::memcmp(in.kx.data(), in.kx.data() + 12 * k, 12 * sizeof(double)) != 0) return false;
    return true;
}

void camera_at(const SceneDesc &sd, double t, DevCamera &out)
{
    // Camera basis in FP64, rounded once to FP32.
    double cam[9];
    keyed(sd.cam.kt, sd.cam.elu, 9, t, cam);
    double f[3] = {cam[3] - cam[0], cam[4] - cam[1], cam[5] - cam[2]};
    const double fl = std::sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    f[0] = f[0] / fl; f[1] = f[1] / fl; f[2] = f[2] / fl;
    const double *up = cam + 6;
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    const double rl = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    r[0] = r[0] / rl; r[1] = r[1] / rl; r[2] = r[2] / rl;
    const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    const double th = std::tan(sd.cam.vfov * (3.14159265358979323846 / 360.0));
    for (int c = 0; c < 3; ++c) {
        out.eye[c] = (float)cam[c];
        out.fwd[c] = (float)f[c];
        out.right[c] = (float)r[c];
        out.up[c] = (float)u[c];
    }
    out.sx = (float)(th * ((double)sd.cam.width / (double)sd.cam.height));
    out.sy = (float)th;
}

float bvh_padding(const SceneDesc &sd, const HostInstant &a, const HostInstant &b)
{
    // Box padding grows with the largest coordinate magnitude of geometry,
    // camera and lights, far above the rounding of the fused slab test.
    float mx = 0.0f;
    for (float v : a.tri) mx = std::max(mx, std::fabs(v));
    for (float v : b.tri) mx = std::max(mx, std::fabs(v));
    // Ray origins on a thin lens lie within its radius of the eye.  The eye
    // moves on straight segments between the camera keys, so the keys bound
    // it at every time: one BVH serves all times of a scene whose instances
    // do not move.
    for (int c = 0; c < 3; ++c) {
        mx = std::max(mx, std::fabs(a.cam.eye[c]) + sd.lens_radius);
        mx = std::max(mx, std::fabs(b.cam.eye[c]) + sd.lens_radius);
    }
    for (size_t k = 0; 9 * k + 2 < sd.cam.elu.size(); ++k)
        for (int c = 0; c < 3; ++c)
            mx = std::max(mx, (float)std::fabs(sd.cam.elu[9 * k + c]) + sd.lens_radius);
    for (float v : sd.pl_pos) mx = std::max(mx, std::fabs(v));
    return std::ldexp(mx + 1.0f, -16);
}

// ---------------------------------------------------------------------------
// FP16 plane offsets.  Offsets from a node's origin are >= 0; they are
// rounded outward to normal IEEE binary16 values or zero (no subnormals, so
// the result does not depend on the device's FP16 denormal mode):
// half_up(x) is the smallest such value >= x, half_down(x) the largest <= x.

static uint16_t half_bits(double v)
{
    // v is zero or a normal binary16 value.
    if (v == 0.0) return 0;
    int e = 0;
    const double f = std::frexp(v, &e);  // v = f 2^e, f in [0.5, 1)
    const uint32_t mant = (uint32_t)std::lround((2.0 * f - 1.0) * 1024.0);
    return (uint16_t)((uint32_t)(e - 1 + 15) << 10 | mant);
}

static uint16_t half_directed(double x, bool up)
{
    if (!(x >= 0.0)) fail(EVRT_E_INVALID, "negative or non-finite FP16 plane offset");
    // (Offsets reach at most 2^15 with the tree's plane scale.)
    if (x < 0x1p-14) return up && x > 0.0 ? half_bits(0x1p-14) : 0;
    int e = 0;
    std::frexp(x, &e);
    const double q = std::ldexp(1.0, e - 11);  // spacing of halves in [2^(e-1), 2^e)
    const double v = (up ? std::ceil(x / q) : std::floor(x / q)) * q;
    if (v > 65504.0) fail(EVRT_E_UNSUPPORTED, "FP16 plane offset out of range");
    return half_bits(v);
}

static double half_value(uint16_t b)
{
    const uint32_t E = (b >> 10) & 0x1fu, mant = b & 0x3ffu;
    const double sign = (b & 0x8000u) ? -1.0 : 1.0;
    if (E == 0x1f) return mant ? NAN : sign * INFINITY;
    if (E == 0) return sign * std::ldexp((double)mant, -24);
    return sign * std::ldexp(1.0 + (double)mant / 1024.0, (int)E - 15);
}

// ---------------------------------------------------------------------------
// Binned SAH binary BVH, collapsed into a 4-wide BVH.

namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const Box &b)
    {
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], b.lo[c]);
            hi[c] = std::max(hi[c], b.hi[c]);
        }
    }
    void grow_pt(const float *p)
    {
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], p[c]);
            hi[c] = std::max(hi[c], p[c]);
        }
    }
    double area() const
    {
        if (!(lo[0] <= hi[0])) return 0.0;
        const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct BNode {
    Box box;
    int32_t child[2] = {-1, -1};   // build-node ids (inner) ...
    uint32_t first = 0, count = 0; // ... or a leaf range (count > 0)
};

struct Builder {
    const std::vector<float> &tri;
    std::vector<Box> tbox;
    std::vector<float> cen;  // [n][3]
    std::vector<uint32_t> ref;
    std::vector<BNode> nodes;

    explicit Builder(const std::vector<float> &t) : tri(t) {}

    static constexpr int kBins = 16;
#ifndef EVRT_LEAF_TARGET
#define EVRT_LEAF_TARGET 4
#endif
    static constexpr uint32_t kLeafTarget = EVRT_LEAF_TARGET;
    static constexpr uint32_t kSahDepthLimit = 32;

    int32_t build(uint32_t b, uint32_t e, uint32_t depth) { return build_into(nodes, b, e, depth); }

    // Subtrees of at least kParallelTris triangles in the top kParallelDepth
    // levels build their left half on another host thread, into a vector of
    // its own appended afterwards (ids shifted); the tree is the same as a
    // serial build's, only its node numbering differs.
    static constexpr uint32_t kParallelTris = 1u << 15;
    static constexpr uint32_t kParallelDepth = 5;
    // Extra builder threads of the whole process at once (instants may be
    // built on several host threads themselves).
    static constexpr int kMaxBuildThreads = 16;
    static std::atomic<int> &build_threads()
    {
        static std::atomic<int> n{0};
        return n;
    }

    int32_t build_into(std::vector<BNode> &nodes, uint32_t b, uint32_t e, uint32_t depth)
    {
        const int32_t id = (int32_t)nodes.size();
        nodes.emplace_back();
        Box bb, cb;
        for (uint32_t i = b; i < e; ++i) {
            bb.grow(tbox[ref[i]]);
            cb.grow_pt(&cen[3 * (size_t)ref[i]]);
        }
        nodes[id].box = bb;
        const uint32_t n = e - b;
        if (n <= kLeafTarget) {
            nodes[id].first = b;
            nodes[id].count = n;
            return id;
        }
        int axis = -1;
        uint32_t mid = b;
        if (depth < kSahDepthLimit) {
            double best = INFINITY;
            int best_axis = -1, best_bin = -1;
            for (int a = 0; a < 3; ++a) {
                const float ext = cb.hi[a] - cb.lo[a];
                if (!(ext > 0.0f)) continue;
                Box bins[kBins];
                uint32_t cnt[kBins] = {0};
                const double scale = kBins / (double)ext;
                for (uint32_t i = b; i < e; ++i) {
                    int k = (int)(((double)cen[3 * (size_t)ref[i] + a] - cb.lo[a]) * scale);
                    k = std::min(std::max(k, 0), kBins - 1);
                    cnt[k]++;
                    bins[k].grow(tbox[ref[i]]);
                }
                double left_area[kBins];
                uint32_t left_cnt[kBins];
                Box acc;
                uint32_t c = 0;
                for (int k = 0; k < kBins - 1; ++k) {
                    acc.grow(bins[k]);
                    c += cnt[k];
                    left_area[k] = acc.area();
                    left_cnt[k] = c;
                }
                acc = Box();
                c = 0;
                for (int k = kBins - 1; k > 0; --k) {
                    acc.grow(bins[k]);
                    c += cnt[k];
                    if (left_cnt[k - 1] == 0 || c == 0) continue;
                    const double cost = left_area[k - 1] * left_cnt[k - 1] + acc.area() * c;
                    if (cost < best) {
                        best = cost;
                        best_axis = a;
                        best_bin = k;
                    }
                }
            }
            const double leaf_cost = bb.area() * n;
            const double split_cost = bb.area() + best;  // one traversal step + children
            if (best_axis >= 0 && (split_cost < leaf_cost || n > kMaxLeafTris)) {
                axis = best_axis;
                const double scale = kBins / (double)(cb.hi[axis] - cb.lo[axis]);
                auto it = std::partition(ref.begin() + b, ref.begin() + e, [&](uint32_t r) {
                    int k = (int)(((double)cen[3 * (size_t)r + axis] - cb.lo[axis]) * scale);
                    k = std::min(std::max(k, 0), kBins - 1);
                    return k < best_bin;
                });
                mid = (uint32_t)(it - ref.begin());
            } else if (best_axis < 0 && n <= kMaxLeafTris) {
                nodes[id].first = b;
                nodes[id].count = n;
                return id;
            } else if (n <= kMaxLeafTris) {
                nodes[id].first = b;
                nodes[id].count = n;
                return id;
            }
        }
        if (mid == b || mid == e) {
            // Object-median split on the widest centroid axis.
            int a = 0;
            for (int c = 1; c < 3; ++c)
                if (cb.hi[c] - cb.lo[c] > cb.hi[a] - cb.lo[a]) a = c;
            mid = b + n / 2;
            std::nth_element(ref.begin() + b, ref.begin() + mid, ref.begin() + e, [&](uint32_t x, uint32_t y) {
                const float cx = cen[3 * (size_t)x + a], cy = cen[3 * (size_t)y + a];
                return cx < cy || (cx == cy && x < y);
            });
        }
        int32_t l, r;
        bool par = false;
        if (n >= kParallelTris && depth < kParallelDepth) {
            if (build_threads().fetch_add(1) < kMaxBuildThreads) par = true;
            else build_threads().fetch_sub(1);
        }
        if (par) {
            std::vector<BNode> left;
            auto fut = std::async(std::launch::async, [this, &left, b, mid, depth] {
                struct Release {
                    ~Release() { build_threads().fetch_sub(1); }
                } release;
                return build_into(left, b, mid, depth + 1);
            });
            r = build_into(nodes, mid, e, depth + 1);
            const int32_t l_local = fut.get();
            const int32_t off = (int32_t)nodes.size();
            for (BNode nd : left) {
                if (nd.count == 0) {
                    nd.child[0] += off;
                    nd.child[1] += off;
                }
                nodes.push_back(nd);
            }
            l = l_local + off;
        } else {
            l = build_into(nodes, b, mid, depth + 1);
            r = build_into(nodes, mid, e, depth + 1);
        }
        nodes[id].child[0] = l;
        nodes[id].child[1] = r;
        return id;
    }
};

inline float pad_down(float v, float pad)
{
    float r = (float)((double)v - (double)pad);
    if ((double)r > (double)v - (double)pad) r = std::nextafter(r, -INFINITY);
    return r;
}

inline float pad_up(float v, float pad)
{
    float r = (float)((double)v + (double)pad);
    if ((double)r < (double)v + (double)pad) r = std::nextafter(r, INFINITY);
    return r;
}

}  // namespace

void build_bvh(HostInstant &h, uint32_t n_lds_max, float pad)
{
    const uint32_t nt = (uint32_t)(h.tri.size() / 9);
    h.nodes.clear();
    h.tris.clear();
    h.root = kEmptyRef;
    h.n_lds = 0;
    h.depth = 0;
    h.sah_cost = 0.0;
    if (nt == 0) return;
    Builder B(h.tri);
    B.tbox.resize(nt);
    B.cen.resize(3 * (size_t)nt);
    B.ref.resize(nt);
    for (uint32_t p = 0; p < nt; ++p) {
        const float *v = &h.tri[9 * (size_t)p];
        Box b;
        for (int k = 0; k < 3; ++k) b.grow_pt(v + 3 * k);
        B.tbox[p] = b;
        for (int c = 0; c < 3; ++c) B.cen[3 * (size_t)p + c] = (float)(((double)v[c] + v[3 + c] + v[6 + c]) / 3.0);
        B.ref[p] = p;
    }
    B.nodes.reserve(2 * (size_t)nt / Builder::kLeafTarget + 16);
    const int32_t broot = B.build(0, nt, 0);

    // Triangles in leaf order.
    h.tris.resize(3 * (size_t)nt);
    for (uint32_t i = 0; i < nt; ++i) {
        const uint32_t p = B.ref[i];
        const float *v = &h.tri[9 * (size_t)p];
        h.tris[3 * (size_t)i + 0] = make_float4(v[0], v[1], v[2], u2f(p));
        h.tris[3 * (size_t)i + 1] = make_float4(v[3], v[4], v[5], 0.0f);
        h.tris[3 * (size_t)i + 2] = make_float4(v[6], v[7], v[8], 0.0f);
    }

    auto leaf_ref = [&](const BNode &n) -> int32_t {
        return (int32_t) ~((n.first << kLeafCountBits) | (n.count - 1));
    };
    // SAH cost of the binary tree (a build-quality statistic).
    double cost = 0.0;
    const double root_area = B.nodes[broot].box.area();
    for (const BNode &n : B.nodes) cost += n.box.area() / root_area * (n.count ? (double)n.count : 1.0);
    h.sah_cost = cost;
    if (B.nodes[broot].count > 0) {
        h.root = leaf_ref(B.nodes[broot]);
        return;
    }
    // 4-wide tree: the children of a wide node are the grandchildren of a
    // binary inner node (a binary child that is a leaf stays itself), so
    // every wide level consumes two binary levels and the wide depth is at
    // most half the binary depth, rounded up.
    auto wide_children = [&](int32_t b, int32_t out[4]) -> int {
        int k = 0;
        for (int c = 0; c < 2; ++c) {
            const int32_t ch = B.nodes[b].child[c];
            if (B.nodes[ch].count) {
                out[k++] = ch;
            } else {
                out[k++] = B.nodes[ch].child[0];
                out[k++] = B.nodes[ch].child[1];
            }
        }
        return k;
    };
    // Wide nodes: breadth-first for the first n_lds_max (the LDS treelet),
    // then each remaining subtree depth-first.
    std::vector<int32_t> order;
    std::vector<int32_t> newid(B.nodes.size(), -1);
    std::vector<uint32_t> wdepth(B.nodes.size(), 0);
    std::vector<int32_t> queue{broot};
    wdepth[broot] = 1;
    size_t qh = 0;
    int32_t ch[4];
    while (qh < queue.size() && order.size() < n_lds_max) {
        const int32_t b = queue[qh++];
        newid[b] = (int32_t)order.size();
        order.push_back(b);
        const int k = wide_children(b, ch);
        for (int i = 0; i < k; ++i)
            if (B.nodes[ch[i]].count == 0) {
                wdepth[ch[i]] = wdepth[b] + 1;
                queue.push_back(ch[i]);
            }
    }
    h.n_lds = (uint32_t)order.size();
    std::vector<int32_t> stack;
    for (size_t q = qh; q < queue.size(); ++q) {
        stack.push_back(queue[q]);
        while (!stack.empty()) {
            const int32_t b = stack.back();
            stack.pop_back();
            newid[b] = (int32_t)order.size();
            order.push_back(b);
            const int k = wide_children(b, ch);
            for (int i = k - 1; i >= 0; --i)
                if (B.nodes[ch[i]].count == 0) {
                    wdepth[ch[i]] = wdepth[b] + 1;
                    stack.push_back(ch[i]);
                }
        }
    }
    h.nodes.assign(8 * order.size(), make_float4(0.0f, 0.0f, 0.0f, 0.0f));
#if EVRT_HALF_NODES
    // One power-of-two scale s = 2^e for the whole tree: origins are stored
    // as origin / s and plane offsets as offset / s, so that the widest node
    // (the root) spans at most 2^15 FP16 units; the kernels scale each ray's
    // reciprocal direction by s once, which leaves every product unchanged.
    // e = 0 unless the scene is wider than 2^15 units.
    int plane_exp = 0;
    {
        const Box &rb = B.nodes[broot].box;
        double ext = 0.0;
        for (int c = 0; c < 3; ++c)
            ext = std::max(ext, (double)pad_up(rb.hi[c], pad) - (double)pad_down(rb.lo[c], pad));
        while (std::ldexp(ext, -plane_exp) > 32768.0) ++plane_exp;
    }
    h.plane_scale = std::ldexp(1.0f, plane_exp);
#endif
    uint32_t depth = 0;
    for (size_t i = 0; i < order.size(); ++i) {
        depth = std::max(depth, wdepth[order[i]]);
        const int k = wide_children(order[i], ch);
        float lo[3][4], hi[3][4];
        uint32_t ref[4];
        for (int j = 0; j < 4; ++j) {
            if (j < k) {
                const BNode &n = B.nodes[ch[j]];
                for (int c = 0; c < 3; ++c) {
                    lo[c][j] = pad_down(n.box.lo[c], pad);
                    hi[c][j] = pad_up(n.box.hi[c], pad);
                }
                ref[j] = (uint32_t)(n.count ? leaf_ref(n) : newid[ch[j]]);
            } else {
                // Empty slot: its near plane is at +inf and its far plane
                // at -inf for either sign of the ray direction.
                for (int c = 0; c < 3; ++c) {
                    lo[c][j] = INFINITY;
                    hi[c][j] = -INFINITY;
                }
                ref[j] = (uint32_t)kEmptySlotRef;
            }
        }
        float4 *o = &h.nodes[8 * i];
#if EVRT_HALF_NODES
        // Row 0: the node's origin (lowest child plane per axis); row 1:
        // references; from byte 32, per axis six words [lo01 lo23 hi01
        // hi23 lo01 lo23]: the children's lower then upper planes as FP16
        // offsets from the origin rounded outward (child 2j in the low half
        // of word j), the lower ones repeated so that one 16 B load at word
        // 0 or 2 returns an axis's near then far planes for either sign of
        // the ray direction; bytes 104-127 zero.
        float org[3];
        for (int c = 0; c < 3; ++c) {
            org[c] = INFINITY;
            for (int j = 0; j < k; ++j) org[c] = std::min(org[c], lo[c][j]);
        }
        float org_s[3];
        for (int c = 0; c < 3; ++c) {
            org_s[c] = std::ldexp(org[c], -plane_exp);
            if (std::ldexp(org_s[c], plane_exp) != org[c]) fail(EVRT_E_UNSUPPORTED, "node origin not exact under the plane scale");
        }
        o[0] = make_float4(org_s[0], org_s[1], org_s[2], 0.0f);
        o[1] = make_float4(u2f(ref[0]), u2f(ref[1]), u2f(ref[2]), u2f(ref[3]));
        float *words = &o[2].x;
        for (int c = 0; c < 3; ++c) {
            uint32_t w[4];
            for (int jj = 0; jj < 2; ++jj) {
                uint16_t lq[2], hq[2];
                for (int b = 0; b < 2; ++b) {
                    const int j = 2 * jj + b;
                    if (j < k) {
                        lq[b] = half_directed(std::ldexp((double)lo[c][j] - (double)org[c], -plane_exp), false);
                        hq[b] = half_directed(std::ldexp((double)hi[c][j] - (double)org[c], -plane_exp), true);
                    } else {
                        lq[b] = kHalfPosInf;
                        hq[b] = kHalfNegInf;
                    }
                }
                w[jj] = (uint32_t)lq[0] | ((uint32_t)lq[1] << 16);
                w[2 + jj] = (uint32_t)hq[0] | ((uint32_t)hq[1] << 16);
            }
            const uint32_t row[6] = {w[0], w[1], w[2], w[3], w[0], w[1]};
            for (int q = 0; q < 6; ++q) words[6 * c + q] = u2f(row[q]);
        }
#else
        for (int c = 0; c < 3; ++c) {
            o[2 * c] = make_float4(lo[c][0], lo[c][1], lo[c][2], lo[c][3]);
            o[2 * c + 1] = make_float4(hi[c][0], hi[c][1], hi[c][2], hi[c][3]);
        }
        o[6] = make_float4(u2f(ref[0]), u2f(ref[1]), u2f(ref[2]), u2f(ref[3]));
#endif
    }
    h.root = 0;
    h.depth = depth;
}

std::string check_bvh(const HostInstant &h, float pad)
{
    const uint32_t nt = (uint32_t)(h.tri.size() / 9);
    if (nt == 0) return h.root == kEmptyRef ? "" : "empty scene with a root";
    std::vector<uint32_t> seen(nt, 0);
    const uint32_t n_nodes = (uint32_t)(h.nodes.size() / 8);
    std::vector<uint32_t> visited(n_nodes, 0);
    // (ref, intersection of the padded boxes of all its ancestors' slots,
    // wide depth of the node that holds it)
    struct Item {
        int32_t ref;
        float lo[3], hi[3];
        uint32_t depth;
    };
    std::vector<Item> st;
    st.push_back(Item{h.root, {-INFINITY, -INFINITY, -INFINITY}, {INFINITY, INFINITY, INFINITY}, 0});
    uint32_t max_depth = 0;
    while (!st.empty()) {
        const Item it = st.back();
        st.pop_back();
        if (it.ref < 0) {
            const uint32_t packed = ~(uint32_t)it.ref;
            const uint32_t first = packed >> kLeafCountBits, count = (packed & (kMaxLeafTris - 1)) + 1;
            if (first + count > nt) return "leaf range out of bounds";
            for (uint32_t k = first; k < first + count; ++k) {
                const float4 *t = &h.tris[3 * (size_t)k];
                const uint32_t p = f2u(t[0].w);
                if (p >= nt) return "bad primitive id";
                seen[p]++;
                const float v[9] = {t[0].x, t[0].y, t[0].z, t[1].x, t[1].y, t[1].z, t[2].x, t[2].y, t[2].z};
                for (int j = 0; j < 9; ++j)
                    if (v[j] != h.tri[9 * (size_t)p + j]) return "leaf triangle differs from the world triangle";
                for (int j = 0; j < 3; ++j)
                    for (int c = 0; c < 3; ++c) {
                        const float x = v[3 * j + c];
                        if (!((double)x - it.lo[c] >= (double)pad * 0.5 && (double)it.hi[c] - x >= (double)pad * 0.5))
                            return "triangle not inside the padded boxes of its ancestors";
                    }
            }
            continue;
        }
        if ((uint32_t)it.ref >= n_nodes) return "node index out of bounds";
        if (visited[it.ref]++) return "node reached twice";
        const uint32_t depth = it.depth + 1;
        max_depth = std::max(max_depth, depth);
        const float4 *n = &h.nodes[8 * (size_t)it.ref];
#if EVRT_HALF_NODES
        // Decode: plane = origin + FP16 offset, exactly in FP64.
        float lo_buf[3][4], hi_buf[3][4];
        const double sc = (double)h.plane_scale;
        const float org[3] = {n[0].x, n[0].y, n[0].z};
        const float *words = &n[2].x;
        for (int c = 0; c < 3; ++c) {
            const float *row = words + 6 * c;
            if (f2u(row[4]) != f2u(row[0]) || f2u(row[5]) != f2u(row[1])) return "repeated lower planes differ";
            for (int j = 0; j < 4; ++j) {
                const uint32_t wl = f2u(row[j >> 1]), wh = f2u(row[2 + (j >> 1)]);
                const uint16_t bl = (uint16_t)((j & 1) ? wl >> 16 : wl & 0xffffu);
                const uint16_t bh = (uint16_t)((j & 1) ? wh >> 16 : wh & 0xffffu);
                // Decoded planes enclose the exact boxes; the FP32 rounding
                // here only tightens the check (up for lo, down for hi).
                const double dl = ((double)org[c] + half_value(bl)) * sc, dh = ((double)org[c] + half_value(bh)) * sc;
                lo_buf[c][j] = bl == kHalfPosInf ? INFINITY : (float)dl;
                hi_buf[c][j] = bh == kHalfNegInf ? -INFINITY : (float)dh;
                if (bl != kHalfPosInf && (double)lo_buf[c][j] < dl) lo_buf[c][j] = std::nextafter(lo_buf[c][j], INFINITY);
                if (bh != kHalfNegInf && (double)hi_buf[c][j] > dh) hi_buf[c][j] = std::nextafter(hi_buf[c][j], -INFINITY);
            }
        }
        const float *lo[3] = {lo_buf[0], lo_buf[1], lo_buf[2]};
        const float *hi[3] = {hi_buf[0], hi_buf[1], hi_buf[2]};
        const float *rf = &n[1].x;
#else
        const float *lo[3] = {&n[0].x, &n[2].x, &n[4].x};
        const float *hi[3] = {&n[1].x, &n[3].x, &n[5].x};
        const float *rf = &n[6].x;
#endif
        int used = 0;
        for (int j = 0; j < 4; ++j) {
            const bool empty = lo[0][j] == INFINITY;
            if (empty) {
                for (int c = 0; c < 3; ++c)
                    if (lo[c][j] != INFINITY || hi[c][j] != -INFINITY) return "empty slot with a box";
                if ((int32_t)f2u(rf[j]) != kEmptySlotRef) return "empty slot with a child";
                continue;
            }
            ++used;
            Item ci{(int32_t)f2u(rf[j]), {0, 0, 0}, {0, 0, 0}, depth};
            for (int c = 0; c < 3; ++c) {
                if (!(lo[c][j] <= hi[c][j])) return "inverted child box";
                ci.lo[c] = std::max(it.lo[c], lo[c][j]);
                ci.hi[c] = std::min(it.hi[c], hi[c][j]);
            }
            st.push_back(ci);
        }
        if (used < 2) return "inner node with fewer than two children";
#if EVRT_HALF_NODES
        if (f2u(n[0].w) != 0u) return "origin row padding not zero";
        for (int q = 26; q < 32; ++q)
            if (f2u((&n[0].x)[q]) != 0u) return "node padding not zero";
#else
        if (n[7].x != 0.0f || n[7].y != 0.0f || n[7].z != 0.0f || n[7].w != 0.0f) return "padding row not zero";
#endif
    }
    for (uint32_t p = 0; p < nt; ++p)
        if (seen[p] != 1) return "primitive missing or duplicated";
    for (uint32_t i = 0; i < n_nodes; ++i)
        if (!visited[i]) return "unreachable node";
    if (max_depth != h.depth) return "recorded depth differs from the tree";
    if (max_depth > (uint32_t)traverse_max_depth()) return "tree deeper than the traversal stack";
    return "";
}

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
}

// ---------------------------------------------------------------------------
// Student t quantile for integer df.  The CDF uses the finite series of
// Abramowitz & Stegun 26.7.3 (odd df) and 26.7.4 (even df) for
// A(t) = P(|T| <= t) in terms of theta = atan(t / sqrt(df)); the quantile
// is found by bisection to full double precision.

static double t_abs_prob(double t, uint32_t df)
{
    const double th = std::atan(t / std::sqrt((double)df));
    const double s = std::sin(th), c = std::cos(th), c2 = c * c;
    if (df % 2 == 1) {
        double sum = 0.0;
        if (df > 1) {
            double term = c;
            sum = c;
            for (uint32_t k = 3; k + 2 <= df; k += 2) {
                term *= c2 * (double)(k - 1) / (double)k;
                sum += term;
            }
        }
        return (2.0 / 3.14159265358979323846) * (th + s * sum);
    }
    double term = 1.0, sum = 1.0;
    for (uint32_t k = 2; k + 2 <= df; k += 2) {
        term *= c2 * (double)(k - 1) / (double)k;
        sum += term;
    }
    return s * sum;
}

static double t_cdf_int(double t, uint32_t df)
{
    const double a = t_abs_prob(std::fabs(t), df);
    return t < 0.0 ? 0.5 - 0.5 * a : 0.5 + 0.5 * a;
}

double t_quantile(double p, uint32_t df)
{
    if (!(p > 0.0) || !(p < 1.0) || df == 0) return NAN;
    if (p == 0.5) return 0.0;
    const bool upper = p > 0.5;
    const double pl = upper ? 1.0 - p : p;  // solve in the lower tail
    double lo = -1.0, hi = 0.0;
    while (t_cdf_int(lo, df) > pl) {
        hi = lo;
        lo *= 2.0;
        if (lo < -1e300) break;
    }
    for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (t_cdf_int(mid, df) < pl) lo = mid;
        else hi = mid;
    }
    const double q = 0.5 * (lo + hi);
    return upper ? -q : q;
}

}  // namespace evrt
