// search.hip -- guides of 2..8 channels (SB_GUIDE_U8XN / SB_GUIDE_U16XN),
// looked up by an exact nearest-texel search instead of a table: the
// additional guiding channels of Sec. 3.1, for which the paper suggests a
// search tree.
//
//   tree build   a k-d tree of the source guide, one level per round of
//                launches.  k_tree_level takes one node per workgroup (its
//                texels are a contiguous run), computes the node's tight box
//                and either makes it a leaf (at most kLeafMax texels, the
//                depth limit, or texels equal in every channel -- then the
//                one of smallest raster index stands for all) or splits the
//                widest element (by weight, then by raw range) at the middle
//                of the box, both sides non-empty, partitioning in one pass
//                into the other texel buffer (left texels from the front,
//                right ones from the back).  k_tree_alloc numbers the next
//                level's nodes in order with a block scan, so the tree is the
//                same on every run.
//   search       depth first, nearer child first; a subtree is skipped only
//                if its box lies strictly farther than the best texel so far
//                (one at equal distance may hold a smaller raster index), so
//                the result is the exact argmin of sum_k w_k (q_k - g_k)^2,
//                ties to the smallest raster index, for any tree shape.
//   k_seeds_n    eight lanes per padded seed record: the seed and its search,
//                the lanes searching disjoint subtrees under a shared bound.
//   k_assign_n   the level loop of Algorithm 2 per pixel (64 x 16 tiles, four
//                rows per thread) with the many-channel error; a pixel no
//                level accepts keeps the nearest candidate its level loop
//                measured.
//   k_fallback_n those pixels' own lookups, one thread per pixel, each search
//                starting from that candidate.
//   k_tree_query the search of caller-given texels (sb_tree_query).
#include <stdio.h>
#include <string.h>

#include <new>
#include <type_traits>

#include "sb_device.h"

namespace sb {
namespace {

constexpr uint32_t kLeafMax = 8;
constexpr int32_t kMaxDepth = 32;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Dword-aligned vectors (node records are 8-byte aligned; global loads need
// dword alignment only).
typedef uint32_t u32x2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Squared distances: 8-bit channels fit 32 bits (8 * 127 * 255^2), 16-bit
// ones need 64 (8 * 127 * 65535^2).
template <int D>
struct DistOf {
  typedef uint32_t type;
};
template <>
struct DistOf<16> {
  typedef uint64_t type;
};

// A texel of S bytes: S / (D / 8) elements of D bits.
template <int S>
struct Tx {
  uint32_t w[S / 4];
};

template <int S>
__device__ __forceinline__ Tx<S> load_tx(const void *base, uint32_t i) {
  Tx<S> t;
  if constexpr (S == 4) {
    t.w[0] = glb(static_cast<const uint32_t *>(base))[i];
  } else if constexpr (S == 8) {
    const u32x2 v = glb(static_cast<const u32x2 *>(base))[i];
    t.w[0] = v.x, t.w[1] = v.y;
  } else {
    const u32x4 v = glb(static_cast<const u32x4 *>(base))[i];
    t.w[0] = v.x, t.w[1] = v.y, t.w[2] = v.z, t.w[3] = v.w;
  }
  return t;
}

template <int S>
__device__ __forceinline__ void store_tx(void *base, uint32_t i, const Tx<S> &t) {
  if constexpr (S == 4) {
    glb(static_cast<uint32_t *>(base))[i] = t.w[0];
  } else if constexpr (S == 8) {
    glb(static_cast<u32x2 *>(base))[i] = u32x2{t.w[0], t.w[1]};
  } else {
    glb(static_cast<u32x4 *>(base))[i] = u32x4{t.w[0], t.w[1], t.w[2], t.w[3]};
  }
}

template <int D, int S>
constexpr int kElems = S * 8 / D;

// Element k (compile-time) of a texel.
template <int D, int S, int K>
__device__ __forceinline__ uint32_t elem(const Tx<S> &t) {
  if constexpr (D == 8) return (t.w[K >> 2] >> ((K & 3) * 8)) & 0xFFu;
  else return (t.w[K >> 1] >> ((K & 1) * 16)) & 0xFFFFu;
}

// Weight of element k: byte k of wn (0 past the guide's channels).
template <int K>
__device__ __forceinline__ uint32_t weight(const uint32_t *wn) {
  return (wn[K >> 2] >> ((K & 3) * 8)) & 0xFFu;
}

// Unrolled loop over the elements k = 0..E-1 with k a compile-time constant.
template <int K, int E, class F>
__device__ __forceinline__ void for_elems(F &&f) {
  if constexpr (K < E) {
    f(std::integral_constant<int, K>());
    for_elems<K + 1, E>(f);
  }
}

// sum_k w_k (a_k - b_k)^2.  |a_k - b_k| < 2^16 fits the 24-bit multiply and
// its square fits 32 bits.
template <int D, int S>
__device__ __forceinline__ typename DistOf<D>::type tx_dist(const Tx<S> &a, const Tx<S> &b,
                                                           const uint32_t *wn) {
  typename DistOf<D>::type d = 0;
  for_elems<0, kElems<D, S>>([&](auto k) {
    constexpr int K = decltype(k)::value;
    const int32_t e = int32_t(elem<D, S, K>(a)) - int32_t(elem<D, S, K>(b));
    const uint32_t e2 = uint32_t(__mul24(e, e));
    if constexpr (D == 8) d += __umul24(e2, weight<K>(wn));
    else d += uint64_t(e2) * weight<K>(wn);
  });
  return d;
}

// The same sum from q to the nearest point of the box [lo, hi].
template <int D, int S>
__device__ __forceinline__ typename DistOf<D>::type box_dist(const Tx<S> &q, const Tx<S> &lo,
                                                            const Tx<S> &hi,
                                                            const uint32_t *wn) {
  typename DistOf<D>::type d = 0;
  for_elems<0, kElems<D, S>>([&](auto k) {
    constexpr int K = decltype(k)::value;
    const uint32_t v = elem<D, S, K>(q), l = elem<D, S, K>(lo), h = elem<D, S, K>(hi);
    const uint32_t e = v < l ? l - v : (v > h ? v - h : 0u);
    const uint32_t e2 = __umul24(e, e);
    if constexpr (D == 8) d += __umul24(e2, weight<K>(wn));
    else d += uint64_t(e2) * weight<K>(wn);
  });
  return d;
}

struct TreeView {
  const void *nodes;
  const void *vals;
  const uint32_t *keys;
};

TreeView tree_view(const void *tree, size_t n, size_t t) {
  const TreeLayout l = tree_layout(n, t);
  const char *b = static_cast<const char *>(tree);
  return TreeView{b + l.nodes, b + l.vals, reinterpret_cast<const uint32_t *>(b + l.keys)};
}

// A node record: box [lo, hi] and link (see tree_layout).
template <int S>
struct Rec {
  Tx<S> lo, hi;
  u32x2 link;
};

template <int S>
__device__ __forceinline__ const SB_GLOBAL unsigned char *rec_at(const void *nodes, uint32_t i) {
  return glb(static_cast<const unsigned char *>(nodes)) + uint64_t(i) * tree_record_bytes(S);
}

template <int S>
__device__ __forceinline__ Rec<S> load_rec(const void *nodes, uint32_t i) {
  const SB_GLOBAL unsigned char *p = rec_at<S>(nodes, i);
  Rec<S> r;
  if constexpr (S == 4) {
    const u32x4a4 v = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(p);
    r.lo.w[0] = v.x, r.hi.w[0] = v.y, r.link = u32x2{v.z, v.w};
  } else if constexpr (S == 8) {
    const u32x4a4 v = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(p);
    const u32x2a4 m = *reinterpret_cast<const SB_GLOBAL u32x2a4 *>(p + 16);
    r.lo.w[0] = v.x, r.lo.w[1] = v.y, r.hi.w[0] = v.z, r.hi.w[1] = v.w, r.link = u32x2{m.x, m.y};
  } else {
    const u32x4a4 a = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(p);
    const u32x4a4 b = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(p + 16);
    const u32x2a4 m = *reinterpret_cast<const SB_GLOBAL u32x2a4 *>(p + 32);
    r.lo.w[0] = a.x, r.lo.w[1] = a.y, r.lo.w[2] = a.z, r.lo.w[3] = a.w;
    r.hi.w[0] = b.x, r.hi.w[1] = b.y, r.hi.w[2] = b.z, r.hi.w[3] = b.w;
    r.link = u32x2{m.x, m.y};
  }
  return r;
}

template <int S>
__device__ __forceinline__ void store_rec_box(void *nodes, uint32_t i, const Tx<S> &lo,
                                              const Tx<S> &hi) {
  SB_GLOBAL uint32_t *p = reinterpret_cast<SB_GLOBAL uint32_t *>(
      const_cast<SB_GLOBAL unsigned char *>(rec_at<S>(nodes, i)));
#pragma unroll
  for (int k = 0; k < S / 4; ++k) p[k] = lo.w[k], p[S / 4 + k] = hi.w[k];
}

__device__ __forceinline__ void store_rec_link(void *nodes, uint32_t rec_bytes, uint32_t i,
                                               u32x2 link) {
  SB_GLOBAL uint32_t *p = reinterpret_cast<SB_GLOBAL uint32_t *>(
      glb(static_cast<unsigned char *>(nodes)) + uint64_t(i) * rec_bytes + (rec_bytes - 8));
  p[0] = link.x;
  p[1] = link.y;
}

// Texels i .. i + kLeafGroup - 1 of the tree's leaves and their keys.
template <int S>
__device__ __forceinline__ void load_group(const TreeView &tv, uint32_t i, Tx<S> *t,
                                           uint32_t *k) {
  static_assert(kLeafGroup == 4, "groups of four texels");
  const SB_GLOBAL u32x4a4 *v = reinterpret_cast<const SB_GLOBAL u32x4a4 *>(
      glb(static_cast<const unsigned char *>(tv.vals)) + uint64_t(i) * S);
  constexpr int W = S / 4;  // words per texel
  u32x4 w[W];
#pragma unroll
  for (int n = 0; n < W; ++n) w[n] = v[n];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < W; ++c) t[m].w[c] = w[(m * W + c) / 4][(m * W + c) % 4];
  const u32x4 kk = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(glb(tv.keys) + i);
  k[0] = kk.x, k[1] = kk.y, k[2] = kk.z, k[3] = kk.w;
}

// A deferred sibling on the search stack: its link and box distance.  For
// 8-bit guides one 8-byte entry, the link packed into a word (inner: the
// first child, < 2^27; leaf: kTreeLeaf | count << 27 | first texel, count
// <= kLeafMax, first texel < 2^26), for 16-bit ones 16 bytes.
template <int D>
struct StackOf {
  typedef u32x4 type;
};
template <>
struct StackOf<8> {
  typedef u32x2 type;
};
template <int D>
__device__ __forceinline__ typename StackOf<D>::type push_entry(u32x2 l,
                                                                typename DistOf<D>::type b) {
  if constexpr (D == 8) {
    const uint32_t w = (l.y & kTreeLeaf) ? (kTreeLeaf | ((l.y & ~kTreeLeaf) << 27) | l.x) : l.x;
    return u32x2{w, b};
  } else {
    return u32x4{l.x, l.y, uint32_t(b), uint32_t(uint64_t(b) >> 32)};
  }
}
template <int D>
__device__ __forceinline__ void pop_entry(const typename StackOf<D>::type &e, u32x2 &l,
                                          typename DistOf<D>::type &b) {
  if constexpr (D == 8) {
    l = u32x2{e.x & 0x07FFFFFFu, (e.x & kTreeLeaf) ? (kTreeLeaf | ((e.x >> 27) & 15u)) : 0u};
    b = e.y;
  } else {
    l = u32x2{e.x, e.y};
    b = typename DistOf<D>::type(e.z) | (typename DistOf<D>::type(e.w) << 32);
  }
}

// The exact lookup of q: the source coordinate x | y << 16 of the texel
// nearest to q under the weights, ties to the smallest raster index (the
// coordinate word y << 16 | x orders like the raster index).  An inner node
// loads both children's records at once (boxes and links), so each level of
// the descent costs one round trip; a deferred sibling is kept with its link
// and its box distance.  The stack holds at most one deferred sibling per
// tree level of the current path, and inner nodes lie above depth
// kMaxDepth - 1.
//
// (best, best_key) may start at a real source texel's distance and
// coordinate (a candidate the caller already measured): every subtree that
// could hold a texel at that distance or nearer is still visited, so the
// result is the same, found with fewer visits.
template <int D, int S>
__device__ uint32_t tree_search(const TreeView &tv, const Tx<S> &q, const uint32_t *wn,
                                typename DistOf<D>::type best = ~typename DistOf<D>::type(0),
                                uint32_t best_key = 0xFFFFFFFFu) {
  typedef typename DistOf<D>::type Dist;
  // one entry per deferred sibling (its link and bound): one scratch store
  // per push and one load per pop, the load issued with a leaf's texels
  // when a leaf comes before the pop
  typename StackOf<D>::type stack[kMaxDepth];
  int32_t sp = 0;
  u32x2 link = load_rec<S>(tv.nodes, 0).link;
  Dist bound = 0;
  for (;;) {
    typename StackOf<D>::type nxt = {};
    if (bound <= best) {
      if (link.y & kTreeLeaf) {
        // the entry popped after this leaf, loaded with the leaf's texels
        if (sp > 0) nxt = stack[sp - 1];
        // the leaf's texels and keys in groups of kLeafGroup, each group's
        // loads issued together (the tree has room past its last entries)
        const uint32_t cnt = link.y & ~kTreeLeaf;
        for (uint32_t j = 0; j < cnt; j += kLeafGroup) {
          Tx<S> t[kLeafGroup];
          uint32_t k[kLeafGroup];
          load_group<S>(tv, link.x + j, t, k);
#pragma unroll
          for (uint32_t m = 0; m < kLeafGroup; ++m) {
            const Dist d = tx_dist<D, S>(q, t[m], wn);
            if (j + m < cnt && (d < best || (d == best && k[m] < best_key)))
              best = d, best_key = k[m];
          }
        }
      } else {
        const Rec<S> r0 = load_rec<S>(tv.nodes, link.x);
        const Rec<S> r1 = load_rec<S>(tv.nodes, link.x + 1);
        const Dist b0 = box_dist<D, S>(q, r0.lo, r0.hi, wn);
        const Dist b1 = box_dist<D, S>(q, r1.lo, r1.hi, wn);
        const bool first0 = b0 <= b1;
        const Dist bf = first0 ? b1 : b0;
        if (bf <= best) {
          const u32x2 fl = first0 ? r1.link : r0.link;
          stack[sp++] = push_entry<D>(fl, bf);
        }
        link = first0 ? r0.link : r1.link;
        bound = first0 ? b0 : b1;
        continue;
      }
    }
    if (sp == 0) break;
    const typename StackOf<D>::type e =
        (link.y & kTreeLeaf) && bound <= best ? nxt : stack[sp - 1];
    --sp;
    pop_entry<D>(e, link, bound);
  }
  return best_key;
}

// v of another lane of the row by the DPP pattern CTRL (every lane of the
// group active).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_from(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_from(uint64_t v) {
  const uint64_t lo = dpp_from<CTRL>(uint32_t(v)), hi = dpp_from<CTRL>(uint32_t(v >> 32));
  return lo | (hi << 32);
}

// The least of v over each aligned group of 8 lanes, in every lane of the
// group (all eight active): pairs within quads (lane ^ 1, lane ^ 2), then
// the group's two quads (lane 7 - i of the group).
template <class T>
__device__ __forceinline__ T group8_min(T v) {
  v = min(v, dpp_from<0xB1>(v));
  v = min(v, dpp_from<0x4E>(v));
  return min(v, dpp_from<0x141>(v));
}

// The same lookup by an aligned group of 8 lanes given the same q: lane g
// of the group searches the subtree reached from the root by the path of
// g's three bits (a leaf met on the way is searched by the one lane whose
// remaining bits are zero), one node per step, and every step prunes with
// the group's best distance so far, which every lane's subtree search may
// use: a subtree farther than a texel any lane has found holds no texel at
// the least distance.  The group's nearest texel, ties to the smallest key,
// is returned to every lane; the subtrees partition the texels, so the
// result is the search's own.
template <int D, int S>
__device__ uint32_t tree_search_group8(const TreeView &tv, const Tx<S> &q, const uint32_t *wn,
                                       uint32_t g) {
  typedef typename DistOf<D>::type Dist;
  Dist best = ~Dist(0), bound = 0;
  uint32_t best_key = 0xFFFFFFFFu;
  u32x2 link = load_rec<S>(tv.nodes, 0).link;
  bool done = false;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (link.y & kTreeLeaf) {
      done = (g >> l) != 0u;
      break;
    }
    const Rec<S> r = load_rec<S>(tv.nodes, link.x + ((g >> l) & 1u));
    link = r.link;
    bound = box_dist<D, S>(q, r.lo, r.hi, wn);
  }
  typename StackOf<D>::type stack[kMaxDepth];
  int32_t sp = 0;
  const uint32_t base = __lane_id() & ~7u;
  for (;;) {
    const Dist gb = group8_min(best);
    if (((__ballot(done) >> base) & 0xFFu) == 0xFFu) break;
    if (done) continue;
    if (bound <= gb) {
      if (link.y & kTreeLeaf) {
        const uint32_t cnt = link.y & ~kTreeLeaf;
        for (uint32_t j = 0; j < cnt; j += kLeafGroup) {
          Tx<S> t[kLeafGroup];
          uint32_t k[kLeafGroup];
          load_group<S>(tv, link.x + j, t, k);
#pragma unroll
          for (uint32_t m = 0; m < kLeafGroup; ++m) {
            const Dist d = tx_dist<D, S>(q, t[m], wn);
            if (j + m < cnt && (d < best || (d == best && k[m] < best_key)))
              best = d, best_key = k[m];
          }
        }
      } else {
        const Rec<S> r0 = load_rec<S>(tv.nodes, link.x);
        const Rec<S> r1 = load_rec<S>(tv.nodes, link.x + 1);
        const Dist b0 = box_dist<D, S>(q, r0.lo, r0.hi, wn);
        const Dist b1 = box_dist<D, S>(q, r1.lo, r1.hi, wn);
        const bool first0 = b0 <= b1;
        const Dist bf = first0 ? b1 : b0;
        if (bf <= gb) stack[sp++] = push_entry<D>(first0 ? r1.link : r0.link, bf);
        link = first0 ? r0.link : r1.link;
        bound = first0 ? b0 : b1;
        continue;
      }
    }
    if (sp == 0) {
      done = true;
      continue;
    }
    --sp;
    pop_entry<D>(stack[sp], link, bound);
  }
  // the group's nearest: least distance, then least key
  const Dist dmin = group8_min(best);
  return group8_min(best == dmin ? best_key : 0xFFFFFFFFu);
}

// ---------------------------------------------------------------- tree build

struct BuildArgs {
  const u32x4 *list_in;  // this level's nodes {first texel, count, node, 0}
  u32x2 *res;            // per list entry {split, texels left of the split}
  const void *vals_in;
  const uint32_t *keys_in;
  void *vals_out;  // the next level's texels (split nodes' children)
  uint32_t *keys_out;
  void *nodes;     // the tree's sections
  void *tvals;
  uint32_t *tkeys;
  uint32_t wn[2];  // build weights (split choice only)
  int32_t channels;
};

template <int S>
__global__ void __launch_bounds__(256) k_tree_init(const void *guide, uint32_t n, uint32_t sw,
                                                   void *vals, uint32_t *keys, u32x4 *list) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    store_tx<S>(vals, i, load_tx<S>(guide, i));
    glb(keys)[i] = ((i / sw) << 16) | (i % sw);
  }
  if (i == 0) glb(list)[0] = u32x4{0u, n, 0u, 0u};
}

// One node per workgroup of NT threads (1024 while the level's nodes are
// large, else 256).
template <int D, int S, int NT>
__global__ void __launch_bounds__(NT) k_tree_level(BuildArgs a, int32_t depth) {
  constexpr int E = kElems<D, S>;
  constexpr uint32_t NW = NT / 64;
  __shared__ uint32_t s_lo[8], s_hi[8], s_key, s_wave[NW];
  const u32x4 ent = glb(a.list_in)[blockIdx.x];
  const uint32_t b = ent.x, c = ent.y, node = ent.z, tid = threadIdx.x;
  if (tid < 8) s_lo[tid] = 0xFFFFFFFFu, s_hi[tid] = 0u;
  if (tid == 0) s_key = 0xFFFFFFFFu;
  __syncthreads();
  // the node's box; four texels per thread in flight
  uint32_t lo[E], hi[E];
#pragma unroll
  for (int k = 0; k < E; ++k) lo[k] = 0xFFFFFFFFu, hi[k] = 0u;
  auto widen = [&](const Tx<S> &t) {
    for_elems<0, E>([&](auto k) {
      constexpr int K = decltype(k)::value;
      lo[K] = min(lo[K], elem<D, S, K>(t));
      hi[K] = max(hi[K], elem<D, S, K>(t));
    });
  };
  uint32_t i = b + tid;
  for (; i + 3 * NT < b + c; i += 4 * NT) {
    const Tx<S> t0 = load_tx<S>(a.vals_in, i), t1 = load_tx<S>(a.vals_in, i + NT);
    const Tx<S> t2 = load_tx<S>(a.vals_in, i + 2 * NT), t3 = load_tx<S>(a.vals_in, i + 3 * NT);
    widen(t0), widen(t1), widen(t2), widen(t3);
  }
  for (; i < b + c; i += NT) widen(load_tx<S>(a.vals_in, i));
  if (tid < c) {
#pragma unroll
    for (int k = 0; k < E; ++k) atomicMin(&s_lo[k], lo[k]), atomicMax(&s_hi[k], hi[k]);
  }
  __syncthreads();
  Tx<S> blo, bhi;
#pragma unroll
  for (int k = 0; k < S / 4; ++k) blo.w[k] = 0u, bhi.w[k] = 0u;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int sh = D == 8 ? (k & 3) * 8 : (k & 1) * 16, wi = D == 8 ? k >> 2 : k >> 1;
    blo.w[wi] |= s_lo[k] << sh;
    bhi.w[wi] |= s_hi[k] << sh;
  }
  if (tid == 0) store_rec_box<S>(a.nodes, node, blo, bhi);
  // the split element: widest by weight, else by raw range; none if every
  // channel is constant over the node
  int32_t ds = -1, dr = -1;
  uint64_t best_w = 0;
  uint32_t best_r = 0;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    if (k >= a.channels) continue;
    const uint32_t r = s_hi[k] - s_lo[k];
    const uint64_t wr = uint64_t(r) * r * ((a.wn[k >> 2] >> ((k & 3) * 8)) & 0xFFu);
    if (wr > best_w) best_w = wr, ds = k;
    if (r > best_r) best_r = r, dr = k;
  }
  if (ds < 0) ds = dr;
  if (ds < 0) {
    // texels equal in every channel: every query sees them at one distance,
    // so the one of smallest raster index stands for all
    uint32_t mk = 0xFFFFFFFFu;
    for (uint32_t i = b + tid; i < b + c; i += NT) mk = min(mk, glb(a.keys_in)[i]);
    if (tid < c) atomicMin(&s_key, mk);
    __syncthreads();
    if (tid == 0) {
      store_tx<S>(a.tvals, b, blo);
      glb(a.tkeys)[b] = s_key;
      store_rec_link(a.nodes, tree_record_bytes(S), node, u32x2{b, 1u | kTreeLeaf});
      glb(a.res)[blockIdx.x] = u32x2{0u, 0u};
    }
    return;
  }
  if (c <= kLeafMax || depth >= kMaxDepth - 1) {
    for (uint32_t i = b + tid; i < b + c; i += NT) {
      store_tx<S>(a.tvals, i, load_tx<S>(a.vals_in, i));
      glb(a.tkeys)[i] = glb(a.keys_in)[i];
    }
    if (tid == 0) {
      store_rec_link(a.nodes, tree_record_bytes(S), node, u32x2{b, c | kTreeLeaf});
      glb(a.res)[blockIdx.x] = u32x2{0u, 0u};
    }
    return;
  }
  // split at s = lo + (hi - lo + 1) / 2: lo < s <= hi, so both sides hold
  // texels (the box is tight).  One pass, NT texels per round: left texels
  // fill [b, b + left) from the front, right ones [b + left, b + c) from the
  // back (the order inside a node does not matter: ties are decided by the
  // stored coordinate), so the left count is known at the end.
  const uint32_t s = s_lo[ds] + (s_hi[ds] - s_lo[ds] + 1) / 2;
  const uint32_t lane = tid & 63u, wave = tid >> 6;
  uint32_t lbase = 0, rbase = 0;
  for (uint32_t base = 0; base < c; base += NT) {
    const uint32_t i = b + base + tid;
    const bool valid = base + tid < c;
    Tx<S> t;
    uint32_t key = 0;
    bool left = false;
    if (valid) {
      t = load_tx<S>(a.vals_in, i);
      key = glb(a.keys_in)[i];
      uint32_t v = 0;
      for_elems<0, E>([&](auto k) {
        constexpr int K = decltype(k)::value;
        if (K == ds) v = elem<D, S, K>(t);
      });
      left = v < s;
    }
    const uint64_t bal = __ballot(left);
    const uint32_t pre =
        __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
    if (lane == 0) s_wave[wave] = uint32_t(__popcll(bal));
    __syncthreads();
    uint32_t woff = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < NW; ++w) {
      woff += w < wave ? s_wave[w] : 0u;
      tot += s_wave[w];
    }
    if (valid) {
      const uint32_t pl = woff + pre;  // left texels before this one in the round
      const uint32_t dst = left ? b + lbase + pl : b + c - 1u - (rbase + (tid - pl));
      store_tx<S>(a.vals_out, dst, t);
      glb(a.keys_out)[dst] = key;
    }
    lbase += tot;
    rbase += min(NT, c - base) - tot;
    __syncthreads();
  }
  if (tid == 0) glb(a.res)[blockIdx.x] = u32x2{1u, lbase};
}

// Numbers the children of this level's split nodes in list order (one
// workgroup of 1024 threads): child pair r of the level gets nodes
// nnodes + 2r, + 2r + 1 and list entries 2r, 2r + 1.  ctr[0] = entries of
// the next level, ctr[1] = nodes so far.
__global__ void __launch_bounds__(1024) k_tree_alloc(const u32x4 *list_in, const u32x2 *res,
                                                     uint32_t m, uint32_t nnodes, u32x4 *list_out,
                                                     void *nodes, uint32_t rec_bytes,
                                                     uint32_t *ctr) {
  __shared__ uint32_t s_wave[16];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  uint32_t run = 0;
  for (uint32_t base = 0; base < m; base += 1024) {
    const uint32_t j = base + tid;
    const bool split = j < m && glb(res)[j].x != 0u;
    const uint64_t bal = __ballot(split);
    const uint32_t pre =
        __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
    if (lane == 0) s_wave[wave] = uint32_t(__popcll(bal));
    __syncthreads();
    uint32_t woff = 0, tot = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      woff += w < wave ? s_wave[w] : 0u;
      tot += s_wave[w];
    }
    if (split) {
      const uint32_t r = run + woff + pre, child = nnodes + 2 * r;
      const u32x4 e = glb(list_in)[j];
      const uint32_t lc = glb(res)[j].y;
      store_rec_link(nodes, rec_bytes, e.z, u32x2{child, 0u});
      glb(list_out)[2 * r] = u32x4{e.x, lc, child, 0u};
      glb(list_out)[2 * r + 1] = u32x4{e.x + lc, e.y - lc, child + 1, 0u};
    }
    run += tot;
    __syncthreads();
  }
  if (tid == 0) {
    glb(ctr)[0] = 2 * run;
    glb(ctr)[1] = nnodes + 2 * run;
  }
}

// ------------------------------------------------------------- frame passes

__device__ inline TreeView frame_tree(const FrameArgs &a) {
  return TreeView{a.t_nodes, a.t_vals, a.t_keys};
}

// Record idx of the padded seed table: the seed of its cell and the
// translation u* - q of the seed's search.
template <int D, int S>
__global__ void __launch_bounds__(256) k_seeds_n(FrameArgs a) {
  // eight lanes per record, each searching part of the tree
  const uint32_t idx = (blockIdx.x * 256 + threadIdx.x) >> 3, g = threadIdx.x & 7u;
  const Levels &lv = a.lv;
  if (idx >= uint32_t(lv.poffset[lv.count])) return;
  int32_t i = 0;
  while (idx >= uint32_t(lv.poffset[i + 1])) ++i;
  const uint32_t local = idx - uint32_t(lv.poffset[i]), pc = uint32_t(lv.cells_x[i] + 2);
  const int32_t cx = int32_t(local % pc) - 1, cy = int32_t(local / pc) - 1;
  const int32_t ls = lv.log2_spacing[i];
  u32x2 rec = {kNoSeed, 0u};
  if (cx >= 0 && cy >= 0 && cx < lv.cells_x[i] && cy < lv.cells_y[i]) {
    const uint32_t j = cell_jitter(a, ls, lv.cells_x[i], lv.offset[i], a.jhash[i], cx, cy);
    const uint32_t sx = (uint32_t(cx) << ls) + (j & 0xFFFFu);
    const uint32_t sy = (uint32_t(cy) << ls) + (j >> 16);
    if (sx < uint32_t(a.w) && sy < uint32_t(a.h)) {
      const uint32_t at = __umul24(sy, uint32_t(a.w)) + sx;
      const uint32_t u =
          tree_search_group8<D, S>(frame_tree(a), load_tx<S>(a.tgt_guide, at), a.wn, g);
      rec.x = pack_xy(4 * sx, 4 * sy);
      rec.y = pack_off(int32_t(u & 0xFFFFu) - int32_t(sx), int32_t(u >> 16) - int32_t(sy));
    }
  }
  if (g == 0) seed_table(a)[idx] = rec;
}

constexpr uint32_t kAssignTW = 64, kAssignTH = 16;

template <int D, int S>
__global__ void __launch_bounds__(256) k_assign_n(FrameArgs a) {
  typedef typename DistOf<D>::type Dist;
  const uint32_t tid = threadIdx.x;
  const uint32_t tiles_x = (uint32_t(a.w) + kAssignTW - 1) / kAssignTW;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int32_t tx0 = int32_t((tile % tiles_x) * kAssignTW);
  const int32_t ty0 = int32_t((tile / tiles_x) * kAssignTH);
  const Levels &lv = a.lv;
  const int32_t L = lv.count;
  const uint32_t sw = uint32_t(a.sw), sh = uint32_t(a.sh);
#pragma unroll 1
  for (int32_t r = 0; r < int32_t(kAssignTH / 4); ++r) {
    const int32_t x = tx0 + int32_t(tid & 63u), y = ty0 + int32_t(tid >> 6) + 4 * r;
    if (x >= a.w || y >= a.h) continue;
    const uint32_t pidx = __umul24(uint32_t(y), uint32_t(a.w)) + uint32_t(x);
    const Tx<S> gt = load_tx<S>(a.tgt_guide, pidx);
    const short2_t p4 = __builtin_bit_cast(short2_t, pack_xy(uint32_t(4 * x), uint32_t(4 * y)));
    bool done = false;
    Dist cd = ~Dist(0);
    uint32_t ckey = 0xFFFFFFFFu;
    for (int32_t i = 0; i < L && !done; ++i) {
      const int32_t ls = lv.log2_spacing[i], pc = lv.cells_x[i] + 2;
      const SB_GLOBAL u32x2 *top = seed_table(a) + lv.poffset[i] + (y >> ls) * pc + (x >> ls);
      int32_t key = INT32_MAX;
#pragma unroll
      for (int32_t k = 0; k < 9; ++k) key = min(key, seed_key(top[(k % 3) * pc + k / 3].x, p4, k));
      if (key == INT32_MAX) continue;
      const int32_t k = key & 15, kx = (k * 11) >> 5;
      const u32x2 rec = top[(k - 3 * kx) * pc + kx];
      const int32_t vx = x + off_x(rec.y), vy = y + off_y(rec.y);
      if (uint32_t(vx) >= sw || uint32_t(vy) >= sh) continue;
      const uint32_t vidx = __umul24(uint32_t(vy), sw) + uint32_t(vx);
      const Dist e = tx_dist<D, S>(gt, load_tx<S>(a.src_guide, vidx), a.wn);
      if (e < a.threshold) {
        glb(a.out_chunk)[pidx] = chunk_code(i, rec.x);
        glb(a.offsets)[pidx] = vote_distance(a, rec.y);
        if (a.out_nnf) glb(a.out_nnf)[pidx] = pack_xy(uint32_t(vx), uint32_t(vy));
        done = true;
      }
      const uint32_t vkey = pack_xy(uint32_t(vx), uint32_t(vy));
      if (e < cd || (e == cd && vkey < ckey)) cd = e, ckey = vkey;
    }
    if (!done) {
      // no level accepts: the fallback code, and in the vote-distance slot
      // the nearest candidate measured (its coordinate, or none), from
      // which k_fallback_n starts the pixel's own search
      glb(a.out_chunk)[pidx] = (uint32_t(L) << 26) | (uint32_t(y) << 13) | uint32_t(x);
      glb(a.offsets)[pidx] = ckey;
    }
  }
}

// The own lookups of the pixels no level accepted (fallback chunk code),
// one thread per pixel of 16 x 16 tiles, each wave an 8 x 8 quarter of its
// tile (neighbours' searches take similar paths and lengths), so a region
// where most pixels fall back has every lane searching once rather than a
// few lanes searching in turn.  The search starts from the candidate the
// level loop left in the vote-distance slot (its distance measured again
// here), then the slot takes the result's vote distance.
template <int D, int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
    k_fallback_n(FrameArgs a) {
  typedef typename DistOf<D>::type Dist;
  const uint32_t tiles_x = (uint32_t(a.w) + 15u) / 16u;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t wq = threadIdx.x >> 6, ln = threadIdx.x & 63u;
  const int32_t x = int32_t((tile % tiles_x) * 16u + (wq & 1u) * 8u + (ln & 7u));
  const int32_t y = int32_t((tile / tiles_x) * 16u + (wq >> 1) * 8u + (ln >> 3));
  if (x >= a.w || y >= a.h) return;
  const uint32_t pidx = __umul24(uint32_t(y), uint32_t(a.w)) + uint32_t(x);
  if ((glb(a.out_chunk)[pidx] >> 26) != uint32_t(a.lv.count)) return;
  const uint32_t ckey = glb(a.offsets)[pidx];
  const Tx<S> gt = load_tx<S>(a.tgt_guide, pidx);
  Dist cd = ~Dist(0);
  if (ckey != 0xFFFFFFFFu) {
    const uint32_t cidx = __umul24(ckey >> 16, uint32_t(a.sw)) + (ckey & 0xFFFFu);
    cd = tx_dist<D, S>(gt, load_tx<S>(a.src_guide, cidx), a.wn);
  }
  const uint32_t u = tree_search<D, S>(frame_tree(a), gt, a.wn, cd, ckey);
  const uint32_t off = pack_off(int32_t(u & 0xFFFFu) - x, int32_t(u >> 16) - y);
  glb(a.offsets)[pidx] = vote_distance(a, off);
  if (a.out_nnf) glb(a.out_nnf)[pidx] = u;
}

template <int D, int S>
__global__ void __launch_bounds__(256) k_tree_query(TreeView tv, const void *q, uint32_t n,
                                                    uint32_t *out, uint32_t w0, uint32_t w1) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t wn[2] = {w0, w1};
  glb(out)[i] = tree_search<D, S>(tv, load_tx<S>(q, i), wn);
}

// ------------------------------------------------------------------- host

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(depth, texel bytes) with both as integral constants for the
// guide's format and texel size.
template <class F>
hipError_t with_format(int32_t fmt, int32_t texel, F &&f) {
  if (fmt == SB_GUIDE_U8XN) {
    if (texel == 4) return f(IC<8>(), IC<4>());
    if (texel == 8) return f(IC<8>(), IC<8>());
  } else if (fmt == SB_GUIDE_U16XN) {
    if (texel == 4) return f(IC<16>(), IC<4>());
    if (texel == 8) return f(IC<16>(), IC<8>());
    if (texel == 16) return f(IC<16>(), IC<16>());
  }
  return hipErrorInvalidValue;
}

unsigned blocks_for(uint64_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

bool side_ok(int32_t v) { return v >= 1 && v <= SB_MAX_SIDE; }

struct BuildWs {
  void *vals[2];
  uint32_t *keys[2];
  u32x4 *list[2];
  u32x2 *res;
  uint32_t *ctr;
  size_t total;
};

BuildWs build_ws(char *base, size_t n, size_t t) {
  BuildWs w;
  size_t at = 0;
  for (int k = 0; k < 2; ++k) {
    w.vals[k] = base ? base + at : nullptr;
    at += align256(n * t);
  }
  for (int k = 0; k < 2; ++k) {
    w.keys[k] = base ? reinterpret_cast<uint32_t *>(base + at) : nullptr;
    at += align256(n * 4);
  }
  for (int k = 0; k < 2; ++k) {
    w.list[k] = base ? reinterpret_cast<u32x4 *>(base + at) : nullptr;
    at += align256(n * 16);
  }
  w.res = base ? reinterpret_cast<u32x2 *>(base + at) : nullptr;
  at += align256(n * 8);
  w.ctr = base ? reinterpret_cast<uint32_t *>(base + at) : nullptr;
  at += 256;
  w.total = at;
  return w;
}

}  // namespace

bool resolve_weights_n(const uint8_t *in, int32_t channels, uint32_t out[2]) {
  out[0] = out[1] = 0u;
  bool any = false;
  for (int32_t k = 0; in && k < channels; ++k) any |= in[k] != 0;
  for (int32_t k = 0; k < channels; ++k) {
    const uint32_t w = any ? in[k] : 1u;
    if (w > 127u) return false;
    out[k >> 2] |= w << ((k & 3) * 8);
  }
  return true;
}

hipError_t launch_search_frame(const FrameArgs &a, hipEvent_t *ev, hipStream_t stream) {
  const uint32_t records = uint32_t(a.lv.poffset[a.lv.count]);
  const uint32_t tiles = ((uint32_t(a.w) + kAssignTW - 1) / kAssignTW) *
                         ((uint32_t(a.h) + kAssignTH - 1) / kAssignTH);
  return with_format(a.fmt, a.texel, [&](auto d, auto s) -> hipError_t {
    constexpr int D = decltype(d)::value, S = decltype(s)::value;
    if (records > 0) k_seeds_n<D, S><<<blocks_for(uint64_t(records) * 8, 256), 256, 0, stream>>>(a);
    if (ev) {
      const hipError_t e = hipEventRecord(ev[1], stream);
      if (e != hipSuccess) return e;
    }
    k_assign_n<D, S><<<tiles, 256, 0, stream>>>(a);
    const uint32_t ftiles = ((uint32_t(a.w) + 15u) / 16u) * ((uint32_t(a.h) + 15u) / 16u);
    k_fallback_n<D, S><<<ftiles, 256, 0, stream>>>(a);
    return hipGetLastError();
  });
}

}  // namespace sb

using namespace sb;

extern "C" {

int32_t sb_texel_bytes(int32_t fmt, int32_t channels) { return search_texel_bytes(fmt, channels); }

size_t sb_tree_bytes(int32_t fmt, int32_t channels, int32_t sw, int32_t sh) {
  const int32_t t = search_texel_bytes(fmt, channels);
  if (t == 0 || !side_ok(sw) || !side_ok(sh)) return 0;
  return tree_layout(size_t(sw) * size_t(sh), size_t(t)).total;
}

size_t sb_tree_workspace_bytes(int32_t fmt, int32_t channels, int32_t sw, int32_t sh) {
  const int32_t t = search_texel_bytes(fmt, channels);
  if (t == 0 || !side_ok(sw) || !side_ok(sh)) return 0;
  return build_ws(nullptr, size_t(sw) * size_t(sh), size_t(t)).total;
}

int sb_tree_build(const void *guide, int32_t fmt, int32_t channels, int32_t sw, int32_t sh,
                  const uint8_t *weights, void *tree, size_t tree_bytes, void *workspace,
                  size_t workspace_bytes, hipStream_t stream) {
  const int32_t t = search_texel_bytes(fmt, channels);
  if (!guide || !tree || !workspace || t == 0 || !side_ok(sw) || !side_ok(sh)) return SB_EINVAL;
  uint32_t wn[2];
  if (!resolve_weights_n(weights, channels, wn)) return SB_EINVAL;
  const uint32_t n = uint32_t(sw) * uint32_t(sh);
  const TreeLayout l = tree_layout(n, size_t(t));
  if (tree_bytes < l.total) return SB_ENOMEM;
  const BuildWs ws = build_ws(static_cast<char *>(workspace), n, size_t(t));
  if (workspace_bytes < ws.total) return SB_ENOMEM;
  char *tb = static_cast<char *>(tree);
  BuildArgs a;
  memset(&a, 0, sizeof a);
  a.nodes = tb + l.nodes;
  a.tvals = tb + l.vals;
  a.tkeys = reinterpret_cast<uint32_t *>(tb + l.keys);
  a.res = ws.res;
  a.wn[0] = wn[0];
  a.wn[1] = wn[1];
  a.channels = channels;
  hipError_t e = with_format(fmt, t, [&](auto d, auto s) -> hipError_t {
    constexpr int D = decltype(d)::value, S = decltype(s)::value;
    k_tree_init<S><<<blocks_for(n, 256), 256, 0, stream>>>(guide, n, uint32_t(sw), ws.vals[0],
                                                          ws.keys[0], ws.list[0]);
    uint32_t m = 1, nnodes = 1;
    int cur = 0;
    for (int32_t depth = 0; m > 0; ++depth) {
      if (depth >= kMaxDepth) return hipErrorUnknown;  // every node at the limit is a leaf
      a.list_in = ws.list[cur];
      a.vals_in = ws.vals[cur];
      a.keys_in = ws.keys[cur];
      a.vals_out = ws.vals[cur ^ 1];
      a.keys_out = ws.keys[cur ^ 1];
      // large nodes (the top levels) take 1024 threads each
      if (uint64_t(m) * 16384u <= uint64_t(n))
        k_tree_level<D, S, 1024><<<m, 1024, 0, stream>>>(a, depth);
      else
        k_tree_level<D, S, 256><<<m, 256, 0, stream>>>(a, depth);
      k_tree_alloc<<<1, 1024, 0, stream>>>(ws.list[cur], ws.res, m, nnodes, ws.list[cur ^ 1],
                                           a.nodes, uint32_t(tree_record_bytes(S)), ws.ctr);
      uint32_t hc[2] = {0u, 0u};
      hipError_t ec = hipMemcpyAsync(hc, ws.ctr, sizeof hc, hipMemcpyDeviceToHost, stream);
      if (ec == hipSuccess) ec = hipStreamSynchronize(stream);
      if (ec != hipSuccess) return ec;
      m = hc[0];
      nnodes = hc[1];
      cur ^= 1;
    }
    // header: nodes, texels, texel bytes, channels (for inspection only)
    uint32_t hdr[4] = {nnodes, n, uint32_t(t), uint32_t(channels)};
    hipError_t ec = hipMemcpyAsync(tb, hdr, sizeof hdr, hipMemcpyHostToDevice, stream);
    if (ec == hipSuccess) ec = hipStreamSynchronize(stream);
    if (ec != hipSuccess) return ec;
    return hipGetLastError();
  });
  if (e != hipSuccess) {
    set_hip_error(e, "sb_tree_build");
    return SB_EHIP;
  }
  return SB_OK;
}

int sb_tree_query(const sb_style *style, const void *queries, int64_t n, uint32_t *out,
                  hipStream_t stream) {
  if (!style || !fmt_search(style->fmt) || !style->tree || !queries || !out || n < 0 ||
      n > int64_t(UINT32_MAX) || !side_ok(style->sw) || !side_ok(style->sh))
    return SB_EINVAL;
  const int32_t t = search_texel_bytes(style->fmt, style->channels);
  uint32_t wn[2];
  if (t == 0 || !resolve_weights_n(style->weights, style->channels, wn)) return SB_EINVAL;
  if (n == 0) return SB_OK;
  const TreeView tv = tree_view(style->tree, size_t(style->sw) * size_t(style->sh), size_t(t));
  hipError_t e = with_format(style->fmt, t, [&](auto d, auto s) -> hipError_t {
    constexpr int D = decltype(d)::value, S = decltype(s)::value;
    k_tree_query<D, S><<<blocks_for(uint64_t(n), 256), 256, 0, stream>>>(tv, queries, uint32_t(n),
                                                                        out, wn[0], wn[1]);
    return hipGetLastError();
  });
  if (e != hipSuccess) {
    set_hip_error(e, "sb_tree_query");
    return SB_EHIP;
  }
  return SB_OK;
}

}  // extern "C"

namespace sb {
// The tree sections a frame of a search-format style reads.
void fill_tree_args(const sb_style *style, FrameArgs *a) {
  const int32_t t = search_texel_bytes(style->fmt, style->channels);
  const TreeView tv = tree_view(style->tree, size_t(style->sw) * size_t(style->sh), size_t(t));
  a->t_nodes = tv.nodes;
  a->t_vals = tv.vals;
  a->t_keys = tv.keys;
  a->texel = t;
  resolve_weights_n(style->weights, style->channels, a->wn);
}
}  // namespace sb
