// Host BVH builder: binned SAH over triangle centroids (binary tree, leaves of at most
// `max_leaf` triangles), then collapsed to a 4-wide tree whose nodes are laid out in
// breadth-first order so that every level is one contiguous range (used by the refit).
//
// The paper builds one acceleration structure per mesh plus a top level over instances
// (Sec. IV-B, "Ray-traced shadows"); this library keeps a single flat BVH over all
// triangles of the scene and refits it when bodies move.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "rc_internal.h"

namespace {

struct Box {
    float lo[3], hi[3];
    void empty()
    {
        for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    }
    void grow(const Box& b)
    {
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], b.lo[k]); hi[k] = std::max(hi[k], b.hi[k]); }
    }
    double area() const
    {
        double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        if (!(dx >= 0) || !(dy >= 0) || !(dz >= 0)) return 0.0;
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct Node2 {
    Box box;
    int32_t left, right;     // -1 for leaves
    uint32_t first, count;   // leaf range in the permuted id array
};

struct Builder {
    const std::vector<Box>* tb;
    const std::vector<float>* cen;   // 3 per triangle
    uint32_t* ids;
    uint32_t bins, max_leaf;
    double node_cost;
    std::vector<Node2> nodes;
    std::atomic<uint32_t> n_nodes{0};

    uint32_t alloc() { return n_nodes.fetch_add(1, std::memory_order_relaxed); }

    uint32_t build(uint32_t b, uint32_t e, int depth)
    {
        uint32_t id = alloc();
        Node2 nd;
        nd.left = nd.right = -1;
        nd.first = b;
        nd.count = e - b;
        nd.box.empty();
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t i = b; i < e; ++i) {
            const Box& t = (*tb)[ids[i]];
            nd.box.grow(t);
            const float* c = &(*cen)[3 * (size_t)ids[i]];
            for (int k = 0; k < 3; ++k) { clo[k] = std::min(clo[k], c[k]); chi[k] = std::max(chi[k], c[k]); }
        }
        uint32_t n = e - b;
        if (n == 1) { nodes[id] = nd; return id; }

        // binned SAH over the three axes
        const int NB = (int)bins;
        double best_cost = INFINITY;
        int best_axis = -1, best_split = -1;
        std::vector<Box> bb(NB);
        std::vector<uint32_t> bc(NB);
        std::vector<double> right_area(NB);
        std::vector<uint32_t> right_cnt(NB);
        for (int axis = 0; axis < 3; ++axis) {
            float ext = chi[axis] - clo[axis];
            if (!(ext > 0.0f)) continue;
            for (int k = 0; k < NB; ++k) { bb[k].empty(); bc[k] = 0; }
            double scale = (double)NB / (double)ext;
            for (uint32_t i = b; i < e; ++i) {
                float c = (*cen)[3 * (size_t)ids[i] + axis];
                int k = (int)(((double)c - clo[axis]) * scale);
                k = std::min(std::max(k, 0), NB - 1);
                bb[k].grow((*tb)[ids[i]]);
                bc[k]++;
            }
            Box acc;
            acc.empty();
            uint32_t cnt = 0;
            for (int k = NB - 1; k > 0; --k) {
                acc.grow(bb[k]);
                cnt += bc[k];
                right_area[k] = acc.area();
                right_cnt[k] = cnt;
            }
            acc.empty();
            cnt = 0;
            for (int k = 0; k < NB - 1; ++k) {
                acc.grow(bb[k]);
                cnt += bc[k];
                if (cnt == 0 || right_cnt[k + 1] == 0) continue;
                double cost = acc.area() * cnt + right_area[k + 1] * right_cnt[k + 1];
                if (cost < best_cost) { best_cost = cost; best_axis = axis; best_split = k + 1; }
            }
        }
        double parea = nd.box.area();
        double split_cost = parea > 0 ? node_cost + best_cost / parea : (double)n;
        if (n <= max_leaf && (best_axis < 0 || (double)n <= split_cost)) { nodes[id] = nd; return id; }

        uint32_t mid;
        if (best_axis < 0) {
            mid = b + n / 2;   // all centroids coincide: split the range in half
        } else {
            double scale = (double)NB / (double)(chi[best_axis] - clo[best_axis]);
            float lo = clo[best_axis];
            int ax = best_axis, sp = best_split;
            uint32_t* m = std::partition(ids + b, ids + e, [&](uint32_t t) {
                int k = (int)(((double)(*cen)[3 * (size_t)t + ax] - lo) * scale);
                k = std::min(std::max(k, 0), NB - 1);
                return k < sp;
            });
            mid = (uint32_t)(m - ids);
            if (mid == b || mid == e) mid = b + n / 2;
        }
        nd.count = 0;
        uint32_t l, r;
        if (n > 100000 && depth < 5) {
            uint32_t lres = 0;
            std::thread th([&] { lres = build(b, mid, depth + 1); });
            r = build(mid, e, depth + 1);
            th.join();
            l = lres;
        } else {
            l = build(b, mid, depth + 1);
            r = build(mid, e, depth + 1);
        }
        nd.left = (int32_t)l;
        nd.right = (int32_t)r;
        nodes[id] = nd;
        return id;
    }
};

void set_child(Node4& n, int slot, const Box& b, uint32_t word)
{
    n.lo_x[slot] = b.lo[0]; n.hi_x[slot] = b.hi[0];
    n.lo_y[slot] = b.lo[1]; n.hi_y[slot] = b.hi[1];
    n.lo_z[slot] = b.lo[2]; n.hi_z[slot] = b.hi[2];
    n.child[slot] = word;
}

}  // namespace

double rc_bvh_sah(const std::vector<Node4>& nodes)
{
    if (nodes.empty()) return 0.0;
    auto area = [](float lx, float hx, float ly, float hy, float lz, float hz) {
        double dx = (double)hx - lx, dy = (double)hy - ly, dz = (double)hz - lz;
        if (!(dx >= 0) || !(dy >= 0) || !(dz >= 0)) return 0.0;
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    };
    const Node4& r = nodes[0];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int c = 0; c < 4; ++c) {
        if (r.child[c] == RC_EMPTY_CHILD) continue;
        lo[0] = std::min(lo[0], r.lo_x[c]); hi[0] = std::max(hi[0], r.hi_x[c]);
        lo[1] = std::min(lo[1], r.lo_y[c]); hi[1] = std::max(hi[1], r.hi_y[c]);
        lo[2] = std::min(lo[2], r.lo_z[c]); hi[2] = std::max(hi[2], r.hi_z[c]);
    }
    double ra = area(lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
    if (ra <= 0) return 0.0;
    double s = 1.0;   // the root itself
    for (const Node4& n : nodes)
        for (int c = 0; c < 4; ++c) {
            uint32_t w = n.child[c];
            if (w == RC_EMPTY_CHILD) continue;
            double a = area(n.lo_x[c], n.hi_x[c], n.lo_y[c], n.hi_y[c], n.lo_z[c], n.hi_z[c]) / ra;
            s += rc_is_leaf(w) ? a * rc_leaf_count(w) : a;
        }
    return s;
}

bool rc_build_bvh_host(const float* pos, const uint32_t* idx, uint32_t n_tris, uint32_t bins,
                       uint32_t max_leaf, float node_cost, HostBvh& out)
{
    out = HostBvh();
    if (n_tris == 0) return false;
    std::vector<Box> tb(n_tris);
    std::vector<float> cen(3 * (size_t)n_tris);
    for (uint32_t t = 0; t < n_tris; ++t) {
        Box b;
        b.empty();
        for (int v = 0; v < 3; ++v) {
            const float* p = pos + 3 * (size_t)idx[3 * (size_t)t + v];
            for (int k = 0; k < 3; ++k) { b.lo[k] = std::min(b.lo[k], p[k]); b.hi[k] = std::max(b.hi[k], p[k]); }
        }
        tb[t] = b;
        for (int k = 0; k < 3; ++k) cen[3 * (size_t)t + k] = 0.5f * b.lo[k] + 0.5f * b.hi[k];
    }
    std::vector<uint32_t> ids(n_tris);
    for (uint32_t t = 0; t < n_tris; ++t) ids[t] = t;

    Builder B;
    B.tb = &tb;
    B.cen = &cen;
    B.ids = ids.data();
    B.bins = bins;
    B.max_leaf = max_leaf;
    B.node_cost = node_cost;
    B.nodes.resize(2 * (size_t)n_tris);
    uint32_t root = B.build(0, n_tris, 0);
    const std::vector<Node2>& N2 = B.nodes;

    // collapse to 4-wide, breadth first
    struct Item { uint32_t n2; uint32_t parent; uint32_t level; };
    std::vector<Item> queue;
    queue.push_back({root, 0xFFFFFFFFu, 0});
    out.nodes.clear();
    out.nodes.reserve(n_tris / 2 + 1);
    uint64_t leaves = 0;
    uint32_t depth = 0;
    for (size_t q = 0; q < queue.size(); ++q) {
        Item it = queue[q];
        Node4 n;
        memset(&n, 0, sizeof(n));
        n.parent = it.parent;
        n.level = it.level;
        depth = std::max(depth, it.level + 1);
        for (int c = 0; c < 4; ++c) {
            n.lo_x[c] = n.lo_y[c] = n.lo_z[c] = INFINITY;
            n.hi_x[c] = n.hi_y[c] = n.hi_z[c] = -INFINITY;
            n.child[c] = RC_EMPTY_CHILD;
        }
        std::vector<uint32_t> kids;
        const Node2& me = N2[it.n2];
        if (me.left < 0) {
            kids.push_back(it.n2);   // a leaf root becomes the single child of the root node
        } else {
            kids.push_back((uint32_t)me.left);
            kids.push_back((uint32_t)me.right);
            while (kids.size() < 4) {
                int pick = -1;
                double best = -1.0;
                for (size_t k = 0; k < kids.size(); ++k) {
                    const Node2& c = N2[kids[k]];
                    if (c.left < 0) continue;
                    double a = c.box.area();
                    if (a > best) { best = a; pick = (int)k; }
                }
                if (pick < 0) break;
                uint32_t open = kids[pick];
                kids[pick] = (uint32_t)N2[open].left;
                kids.insert(kids.begin() + pick + 1, (uint32_t)N2[open].right);
            }
        }
        for (size_t k = 0; k < kids.size(); ++k) {
            const Node2& c = N2[kids[k]];
            if (c.left < 0) {
                set_child(n, (int)k, c.box, rc_make_leaf(c.first, c.count));
                leaves++;
            } else {
                uint32_t child_index = (uint32_t)queue.size();
                queue.push_back({kids[k], (uint32_t)q, it.level + 1});
                set_child(n, (int)k, c.box, child_index);
            }
        }
        out.nodes.push_back(n);
    }
    out.level_start.assign(depth + 1, (uint32_t)out.nodes.size());
    for (size_t i = out.nodes.size(); i-- > 0;) out.level_start[out.nodes[i].level] = (uint32_t)i;
    out.tri_order = ids;
    out.depth = depth;
    out.max_stack = 3 * depth + 1;
    out.n_leaves = leaves;
    out.sah_cost = rc_bvh_sah(out.nodes);
    return true;
}
