// Bounding volume hierarchy for closest-point queries (Algorithm 1,
// DistanceToBoundary).  Host builder and the device layout it produces.
//
// Layout (one "pair node" per internal node): a node stores, for BOTH of its
// children, an axis-aligned box and an oriented slab {y : |n.y - o| <= t},
// plus the two child references, so one node fetch decides which children to
// enter.  The distance lower bound of a child is the larger of the point-box
// and point-slab distances; for a smooth boundary the slab thickness t is
// the sagitta of the child's patch, so the bound is nearly exact in the
// direction of the normal, where axis-aligned boxes are loosest.
// A node is node_scalars(D) scalars:
//   [ lo0[D] hi0[D] lo1[D] hi1[D] | n0[D] o0 t0 | n1[D] o1 t1 | refs ]
//   (2D: 20 scalars, 3D: 24; FP32 nodes are 80 B / 96 B)
// A child reference r >= 0 is another pair node; r < 0 encodes a leaf,
// v = -1 - r: primitives [v >> 3, (v >> 3) + (v & 7) + 1) in leaf order.
// Primitives are stored in leaf order (prim_scalars(D) scalars each: 2D a,b;
// 3D a,b,c padded to 12) with their original indices alongside.
#pragma once
#include <cstdint>
#include <vector>

namespace dwos {

// Largest leaf (primitives per leaf, <= 8: 3-bit count), per dimension.
// Measured with the walk kernels on the 200,000-triangle icosphere
// (65536 points x 1024 walks): leaves of up to 8 triangles 124 / 140 ms
// (forward / differential launch), 6: 121 / 137, 4: 119 / 136; on 2D
// polylines leaves of 8 segments took the star's launches from 22.0 / 29.2
// to 18.4 / 25.0 ms against smaller leaves.
#ifndef DWOS_LEAF_MAX_2D
#define DWOS_LEAF_MAX_2D 8
#endif
#ifndef DWOS_LEAF_MAX_3D
#define DWOS_LEAF_MAX_3D 4
#endif
#ifndef DWOS_STACK_SIZE
#define DWOS_STACK_SIZE 48
#endif
constexpr int kLeafMax2 = DWOS_LEAF_MAX_2D;
constexpr int kLeafMax3 = DWOS_LEAF_MAX_3D;
constexpr int leaf_max(int D) { return D == 2 ? kLeafMax2 : kLeafMax3; }
constexpr int kStackSize = DWOS_STACK_SIZE; // traversal stack entries
constexpr int kMaxDepth = kStackSize - 2;   // builder guarantee (stack never overflows)
static_assert(kLeafMax2 >= 1 && kLeafMax2 <= 8 && kLeafMax3 >= 1 && kLeafMax3 <= 8,
              "leaf size must fit the 3-bit count");

constexpr int node_scalars(int D) { return D == 2 ? 20 : 24; }
constexpr int slab_offset(int D) { return 4 * D; }                  // n0[D] o0 t0 n1[D] o1 t1
constexpr int ref_offset(int D) { return 4 * D + 2 * (D + 2); }     // two int32 child refs
constexpr int prim_scalars(int D) { return D == 2 ? 4 : 12; }

// Padding added to a slab half-thickness so that the rounding of the
// working-precision projection n.x - o can never make the slab bound exceed
// the true distance: 16 units of roundoff of the projected magnitudes.
template <class T>
inline T slab_pad_host(T scale) { return T(16) * (sizeof(T) == 4 ? T(5.9604644775390625e-08) : T(1.1102230246251565e-16)) * scale; }

inline int32_t leaf_ref(int32_t start, int32_t count) { return -1 - ((start << 3) | (count - 1)); }

struct HostNode {
    double lo[2][3];
    double hi[2][3];
    double n[2][3];          // slab normals
    double o[2], t[2];       // slab offsets and half-thicknesses
    int32_t child[2];
    int32_t range[2][2];     // leaf-order primitive range under each child
    int32_t depth;
};

struct HostBVH {
    std::vector<HostNode> nodes;     // nodes[0] is the root
    std::vector<int32_t> order;      // leaf position -> original primitive index
    std::vector<int32_t> leaf_of;    // original primitive -> leaf position
    int max_depth = 0;
};

// Binned-SAH build over primitive bounding boxes.  V: nv x D vertices,
// prims: np x D indices; leaves of at most leaf_max(D) primitives.  Depth is
// kept <= kMaxDepth by switching to median splits when a subtree would
// otherwise get too deep.
HostBVH build_bvh(const double* V, const int32_t* prims, int64_t np, int D);

// Renumber the pair nodes in breadth-first order (root first, then each
// level), so that the top levels of the tree form a prefix of the node array
// that can be staged in LDS.
void reorder_bfs(HostBVH& bvh);


}  // namespace dwos
