// Bounding volume hierarchy for closest-point queries (Algorithm 1,
// DistanceToBoundary).  Host builder and the device layout it produces.
//
// Layout (one "pair node" per internal node): a node stores the bounding
// boxes of BOTH of its children and the two child references, so one node
// fetch decides which children to enter.  A node is NODE_T(D) scalars:
//   [ lo0[D] hi0[D] lo1[D] hi1[D] | refs ]   (3D FP32: 64 B, 2D FP32: 48 B)
// A child reference r >= 0 is another pair node; r < 0 encodes a leaf,
// v = -1 - r: primitives [v >> 3, (v >> 3) + (v & 7) + 1) in leaf order.
// Primitives are stored in leaf order (PRIM_T(D) scalars each: 2D a,b;
// 3D a,b,c padded to 12) with their original indices alongside.
#pragma once
#include <cstdint>
#include <vector>

namespace dwos {

constexpr int kLeafMax = 4;     // primitives per leaf (fits the 3-bit count)
constexpr int kMaxDepth = 40;   // builder guarantee; traversal stack size
constexpr int kStackSize = 48;

constexpr int node_scalars(int D) { return 4 * D + 4; }   // 16 (3D) or 12 (2D)
constexpr int prim_scalars(int D) { return D == 2 ? 4 : 12; }

inline int32_t leaf_ref(int32_t start, int32_t count) { return -1 - ((start << 3) | (count - 1)); }

struct HostNode {
    double lo[2][3];
    double hi[2][3];
    int32_t child[2];
    int32_t depth;
};

struct HostBVH {
    std::vector<HostNode> nodes;     // nodes[0] is the root
    std::vector<int32_t> order;      // leaf position -> original primitive index
    std::vector<int32_t> leaf_of;    // original primitive -> leaf position
    int max_depth = 0;
};

// Binned-SAH build over primitive bounding boxes.  V: nv x D vertices,
// prims: np x D indices.  Depth is kept <= kMaxDepth by switching to
// median splits when a subtree would otherwise get too deep.
HostBVH build_bvh(const double* V, const int32_t* prims, int64_t np, int D);

// Refit order: node indices grouped by depth (deepest level first).
void refit_levels(const HostBVH& bvh, std::vector<int32_t>& order, std::vector<int32_t>& level_start);

}  // namespace dwos
