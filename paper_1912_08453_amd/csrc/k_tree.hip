// Final step without searches for an acyclic template whose labels are
// unique except for one pair of template vertices a, b (kernels of libpm,
// gfx950).
//
// A map of such a template is injective unless it puts a and b on one
// vertex (two vertices of different labels never share an image), so the
// matches are the label-preserving homomorphisms with phi(a) != phi(b).
// At the LCC fixpoint (the coverage rule of the local constraint check)
// every role has a supporting neighbour for each template neighbour; on a
// tree this arc consistency makes every role of omega part of some
// homomorphism, and any homomorphism of the path p_0 = a .. p_k = b
// (each p_i on a vertex holding role p_i) extends to the whole template.
// Hence, with SL_i(u) the images of a over the homomorphisms of p_0..p_i
// that put p_i on u and SR_i(u) the images of b over those of p_i..p_k,
//   role p_i of u is in a match  iff  some x in SL_i(u), y in SR_i(u) differ,
// which a (smallest, largest) summary of each set decides: it fails only
// when both sets are the same single vertex.  A role r off the path, whose
// neighbour towards the path is r', is in a match iff u has a neighbour
// holding r' in a match (the part of the template beyond r is replaced
// without touching a or b).  An edge is in the complete set iff it can
// carry a template edge: a path edge (p_i, p_{i+1}) on (u, w) needs
// SL_i(u) and SR_{i+1}(w) to offer two different vertices, an off-path
// edge (r, r') on (u, w) needs the role r' of w to be in a match.
//
// Summaries are int2 (smallest, largest vertex id; empty: INT32_MAX, -1)
// per side (left, right), path position and active-list position:
// sum[(side * (k + 1) + i) * nA + t].  The sweeps run one thread per
// compacted entry (entries of one row are consecutive, so a wavefront
// reduces each row's share with a segmented scan and one atomic per row
// and array), which keeps hub rows balanced.
#include "device_util.h"
#include "pm_internal.h"

namespace pm {

namespace {

constexpr int kTreeBlock = 256;
constexpr int kEmptyLo = INT32_MAX;
constexpr int kEmptyHi = -1;

__device__ __forceinline__ int2 empty2() { return make_int2(kEmptyLo, kEmptyHi); }

__device__ __forceinline__ bool nonempty(int2 s) { return s.x <= s.y; }

// Two non-empty endpoint sets offer distinct vertices unless both are the
// same single vertex.
__device__ __forceinline__ bool distinct_ends(int2 l, int2 r) {
    return nonempty(l) && nonempty(r) && !(l.x == l.y && r.x == r.y && l.x == r.x);
}

__device__ __forceinline__ int2 merge2(int2 a, int2 b) {
    return make_int2(min(a.x, b.x), max(a.y, b.y));
}

__device__ __forceinline__ int2 *slot(int2 *sum, int64_t nA, int k, int side, int i, int64_t t) {
    return sum + ((int64_t)(side * (k + 1) + i)) * nA + t;
}

// Grid-stride walk over wavefront-aligned chunks of 64 consecutive entries.
#define TREE_FOR_CHUNKS(c_m, e)                                                             \
    for (int64_t base_ = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u));         \
         base_ < (c_m); base_ += (int64_t)gridDim.x * blockDim.x)                           \
        if (const int64_t e = base_ + lane_id(); true)

__global__ __launch_bounds__(kTreeBlock) void tree_pos_kernel(const int32_t *A, int64_t nA,
                                                              int32_t *pos) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nA;
         t += (int64_t)gridDim.x * blockDim.x)
        pos[A[t]] = (int32_t)t;
}

// Every summary empty, then SL_0(u) = {u} for role a, SR_k(u) = {u} for b.
template <typename M>
__global__ __launch_bounds__(kTreeBlock) void tree_init_kernel(const int32_t *A, int64_t nA,
                                                               const M *om, TreePlan tp,
                                                               int2 *sum) {
    const int k = tp.k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nA;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = A[t];
        const uint64_t o = (uint64_t)om[v];
        for (int side = 0; side < 2; ++side)
            for (int i = 0; i <= k; ++i) *slot(sum, nA, k, side, i, t) = empty2();
        if ((o >> tp.path[0]) & 1ull) *slot(sum, nA, k, 0, 0, t) = make_int2(v, v);
        if ((o >> tp.path[k]) & 1ull) *slot(sum, nA, k, 1, k, t) = make_int2(v, v);
    }
}

// Step s of both sweeps: SL_s from SL_{s-1} of the neighbours holding
// p_{s-1}, and SR_{k-s} from SR_{k-s+1} of those holding p_{k-s+1}.
template <typename M>
__global__ __launch_bounds__(kTreeBlock) void tree_sweep_kernel(
    int64_t c_m, const int32_t *__restrict__ c_own, const int32_t *__restrict__ c_col,
    const M *__restrict__ om, const int32_t *__restrict__ pos, TreePlan tp, int s, int2 *sum,
    int64_t nA) {
    const int k = tp.k;
    const int li = s, ri = k - s;
    const int pl = tp.path[li], plp = tp.path[li - 1];
    const int pr = tp.path[ri], prn = tp.path[ri + 1];
    const int lane = lane_id();
    TREE_FOR_CHUNKS(c_m, e) {
        int32_t u = -1;
        int2 l = empty2(), r = empty2();
        if (e < c_m) {
            u = c_own[e];
            const uint64_t ou = (uint64_t)om[u];
            const bool wl = (ou >> pl) & 1ull, wr = (ou >> pr) & 1ull;
            if (wl || wr) {
                const int32_t w = c_col[e];
                const uint64_t ow = (uint64_t)om[w];
                const bool gl = wl && ((ow >> plp) & 1ull), gr = wr && ((ow >> prn) & 1ull);
                if (gl || gr) {
                    // a vertex holding a role is on the active list
                    const int64_t tw = pos[w];
                    if ((uint64_t)tw < (uint64_t)nA) {
                        if (gl) l = *slot(sum, nA, k, 0, li - 1, tw);
                        if (gr) r = *slot(sum, nA, k, 1, ri + 1, tw);
                    }
                }
            }
        }
        if (ballot64(nonempty(l) || nonempty(r)) == 0) continue;
        // segmented reduction over the lanes of one row (keys ascend)
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t ku = __shfl_up(u, off);
            const int lx = __shfl_up(l.x, off), ly = __shfl_up(l.y, off);
            const int rx = __shfl_up(r.x, off), ry = __shfl_up(r.y, off);
            if (lane >= off && ku == u) {
                l = merge2(l, make_int2(lx, ly));
                r = merge2(r, make_int2(rx, ry));
            }
        }
        const int32_t next_u = __shfl_down(u, 1);
        const bool last = lane == 63 || next_u != u;
        const int64_t tu = last && u >= 0 ? pos[u] : -1;
        if ((uint64_t)tu < (uint64_t)nA && (nonempty(l) || nonempty(r))) {
            if (nonempty(l)) {
                int2 *d = slot(sum, nA, k, 0, li, tu);
                atomicMin(&d->x, l.x);
                atomicMax(&d->y, l.y);
            }
            if (nonempty(r)) {
                int2 *d = slot(sum, nA, k, 1, ri, tu);
                atomicMin(&d->x, r.x);
                atomicMax(&d->y, r.y);
            }
        }
    }
}

// Path roles in a match (sat zeroed by the caller).
template <typename M>
__global__ __launch_bounds__(kTreeBlock) void tree_path_kernel(const int32_t *A, int64_t nA,
                                                               const M *om, TreePlan tp,
                                                               const int2 *sum, M *sat) {
    const int k = tp.k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nA;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = A[t];
        const uint64_t o = (uint64_t)om[v];
        uint64_t good = 0;
        for (int i = 0; i <= k; ++i) {
            const int q = tp.path[i];
            if (!((o >> q) & 1ull)) continue;
            const int2 l = sum[((int64_t)i) * nA + t];
            const int2 r = sum[((int64_t)(k + 1 + i)) * nA + t];
            if (distinct_ends(l, r)) good |= 1ull << q;
        }
        if (good) sat[v] = (M)good;
    }
}

// Off-path roles at distance d from the path: role r of u is in a match iff
// a neighbour holds r's neighbour towards the path in a match.
template <typename M>
__global__ __launch_bounds__(kTreeBlock) void tree_branch_kernel(
    int64_t c_m, const int32_t *__restrict__ c_own, const int32_t *__restrict__ c_col,
    const M *__restrict__ om, TreePlan tp, int d, M *sat) {
    const uint64_t dm = tp.depmask[d];
    const int lane = lane_id();
    TREE_FOR_CHUNKS(c_m, e) {
        int32_t u = -1;
        uint64_t bits = 0;
        if (e < c_m) {
            u = c_own[e];
            uint64_t cand = (uint64_t)om[u] & dm;
            if (cand) {
                const uint64_t sw = (uint64_t)sat[c_col[e]];
                while (cand) {
                    const int r = __builtin_ctzll(cand);
                    cand &= cand - 1;
                    if ((sw >> tp.par[r]) & 1ull) bits |= 1ull << r;
                }
            }
        }
        if (ballot64(bits != 0) == 0) continue;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t ku = __shfl_up(u, off);
            const uint64_t b = ((uint64_t)(uint32_t)__shfl_up((int)(uint32_t)(bits >> 32), off) << 32) |
                               (uint32_t)__shfl_up((int)(uint32_t)bits, off);
            if (lane >= off && ku == u) bits |= b;
        }
        const int32_t next_u = __shfl_down(u, 1);
        const bool last = lane == 63 || next_u != u;
        if (last && u >= 0 && bits) atomic_or_elem<M>(sat, u, bits);
    }
}

// Edge output: the entry u -> w is set iff it can carry a template edge of
// some match (both directions of an edge reach the same answer).  Entries
// go by wavefront-aligned chunks, so the bits of a chunk (ascending within
// each row, rows in vertex order) are set with one atomic per output word.
template <typename M>
__device__ __forceinline__ bool tree_edge_good(int32_t u, int32_t w, uint64_t ou,
                                               const M *__restrict__ om,
                                               const int32_t *__restrict__ pos,
                                               const TreePlan &tp, const int2 *__restrict__ sum,
                                               int64_t nA, const M *__restrict__ sat) {
    const int k = tp.k;
    const uint64_t ow = (uint64_t)om[w];
    if (!ow) return false;
    // the certified role sets and list positions are gathered only for
    // the template edges the entry can carry
    for (int j = 0; j < tp.m0; ++j) {
        for (int o = 0; o < 2; ++o) {
            const int x = o ? tp.eb[j] : tp.ea[j];   // on u
            const int y = o ? tp.ea[j] : tp.eb[j];   // on w
            if (!((ou >> x) & 1ull) || !((ow >> y) & 1ull)) continue;
            const int px = tp.pos[x], py = tp.pos[y];
            bool good;
            if (px >= 0 && py >= 0) {
                // path edge: the left part ends on the lower position
                const int64_t tu = pos[u], tw = pos[w];
                if ((uint64_t)tu >= (uint64_t)nA || (uint64_t)tw >= (uint64_t)nA) continue;
                int2 l, r;
                if (py == px + 1) {
                    l = sum[((int64_t)px) * nA + tu];
                    r = sum[((int64_t)(k + 1 + py)) * nA + tw];
                } else {
                    l = sum[((int64_t)py) * nA + tw];
                    r = sum[((int64_t)(k + 1 + px)) * nA + tu];
                }
                good = distinct_ends(l, r);
            } else if (tp.par[x] == y) {
                good = ((uint64_t)sat[w] >> y) & 1ull;   // x off the path, y towards it
            } else {
                good = ((uint64_t)sat[u] >> x) & 1ull;   // y off the path, x towards it
            }
            if (good) return true;
        }
    }
    return false;
}

template <typename M>
__global__ __launch_bounds__(kTreeBlock) void tree_edges_kernel(
    int64_t c_m, const int32_t *__restrict__ c_own, const int32_t *__restrict__ c_col,
    const int32_t *__restrict__ c_off, const int64_t *__restrict__ rp, const M *__restrict__ om,
    const int32_t *__restrict__ pos, TreePlan tp, const int2 *__restrict__ sum, int64_t nA,
    const M *__restrict__ sat, uint64_t *edge_bits) {
    TREE_FOR_CHUNKS(c_m, e) {
        bool good = false;
        int64_t bit = 0;
        if (e < c_m) {
            const int32_t u = c_own[e];
            const uint64_t ou = (uint64_t)om[u];
            if (ou && tree_edge_good<M>(u, c_col[e], ou, om, pos, tp, sum, nA, sat)) {
                good = true;
                bit = rp[u] + c_off[e];
            }
        }
        set_bits_wave(edge_bits, bit, good);
    }
}

int64_t grid_for(int64_t items, int64_t cap) {
    int64_t g = (items + kTreeBlock - 1) / kTreeBlock;
    return std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

template <typename M>
void launch_tree_exact(hipStream_t s, const int32_t *A, int64_t nA, const M *om,
                       int64_t c_m, const int32_t *c_own, const int32_t *c_col,
                       const int32_t *c_off, const int64_t *rp, const TreePlan &tp,
                       int32_t *pos, int2 *sum, M *sat, uint64_t *edge_bits) {
    if (nA <= 0) return;
    const dim3 blk(kTreeBlock);
    const unsigned gv = (unsigned)grid_for(nA, 16384);
    const unsigned ge = (unsigned)grid_for(c_m, 65536);
    hipLaunchKernelGGL(tree_pos_kernel, dim3(gv), blk, 0, s, A, nA, pos);
    hipLaunchKernelGGL(tree_init_kernel<M>, dim3(gv), blk, 0, s, A, nA, om, tp, sum);
    if (c_m > 0)
        for (int st = 1; st <= tp.k; ++st)
            hipLaunchKernelGGL(tree_sweep_kernel<M>, dim3(ge), blk, 0, s, c_m, c_own, c_col, om,
                               pos, tp, st, sum, nA);
    hipLaunchKernelGGL(tree_path_kernel<M>, dim3(gv), blk, 0, s, A, nA, om, tp, sum, sat);
    if (c_m > 0) {
        for (int d = 1; d <= tp.depth; ++d)
            hipLaunchKernelGGL(tree_branch_kernel<M>, dim3(ge), blk, 0, s, c_m, c_own, c_col, om,
                               tp, d, sat);
        if (edge_bits)
            hipLaunchKernelGGL(tree_edges_kernel<M>, dim3(ge), blk, 0, s, c_m, c_own, c_col,
                               c_off, rp, om, pos, tp, sum, nA, sat, edge_bits);
    }
}

#define PM_INSTANTIATE_TREE(M)                                                                   \
    template void launch_tree_exact<M>(hipStream_t, const int32_t *, int64_t, const M *, int64_t, \
                                       const int32_t *, const int32_t *, const int32_t *,         \
                                       const int64_t *, const TreePlan &, int32_t *, int2 *, M *, \
                                       uint64_t *);

PM_INSTANTIATE_TREE(uint8_t)
PM_INSTANTIATE_TREE(uint16_t)
PM_INSTANTIATE_TREE(uint32_t)
PM_INSTANTIATE_TREE(uint64_t)

}  // namespace pm
