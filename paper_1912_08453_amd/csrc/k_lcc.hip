// Local constraint checking kernels for gfx950: role initialisation, degree
// binning with wavefront prefix-sum compaction, the LCC sweep, the
// candidate-subgraph compaction (edge elimination) and a device-wide scan.
//
// LCC (the paper's LCC algorithm and its visitor): a vertex v keeps role q
// iff every template neighbour of q is a role of some neighbour of v
// (coverage) and, for every label L, at least as many distinct neighbours of
// label L carry a role adjacent to q as q has template neighbours of label L
// (distinct-count rule).  The visitor's alive messages become gathers of the
// neighbours' role masks straight from HBM; an edge counts only when the two
// role sets are adjacent in G0, which is exactly what the coverage and count
// tests read, so the edge state is derived and never stored.  Updates are
// made in place: the local rule is monotone in the neighbours' role sets and
// only ever removes roles, so in-place (chaotic) sweeps reach the same
// greatest fixpoint as synchronous sweeps.
#include "device_util.h"
#include "pm_internal.h"

namespace pm {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- helpers
template <typename M>
__device__ __forceinline__ uint64_t reach_of(uint64_t w, const LccTable &tab) {
    uint64_t r = 0;
    for (int q = 0; q < tab.n0; ++q)
        if ((w >> q) & 1ull) r |= tab.adj[q];
    return r;
}

template <bool CNT>
__device__ __forceinline__ uint64_t evaluate(uint64_t w, uint64_t cover, const int *cnt,
                                             const LccTable &tab) {
    uint64_t nw = w;
    if (tab.any) {
        // candidate-set rule: some template neighbour of q is covered
        for (int q = 0; q < tab.n0; ++q)
            if (((w >> q) & 1ull) && !(tab.adj[q] & cover)) nw &= ~(1ull << q);
        return nw;
    }
    for (int q = 0; q < tab.n0; ++q)
        if (((w >> q) & 1ull) && (tab.adj[q] & ~cover)) nw &= ~(1ull << q);
    if constexpr (CNT) {
#pragma unroll
        for (int c = 0; c < kMaxCount; ++c)
            if (c < tab.ncount && ((w >> tab.cq[c]) & 1ull) && cnt[c] < tab.cneed[c])
                nw &= ~(1ull << tab.cq[c]);
    }
    return nw;
}

// Accumulate coverage (OR of the neighbours' role masks) and distinct-count
// tallies over the entries k = k0, k0 + stride, ... < e.  The column ids of
// kUnroll entries are loaded (streaming, non-temporal) before their role
// masks are gathered, so each wavefront keeps several loads in flight.
constexpr int kUnroll = 8;

// With FILT, a bitmap of the vertices whose initial role set is not empty
// (512 KB at 2^22 vertices, resident in L2) is tested first and only those
// role masks are gathered: in the first sweep most neighbours are inactive.
template <typename M, bool CNT, bool FILT = false>
__device__ __forceinline__ void accumulate(const int32_t *__restrict__ col, const M *omega,
                                           int64_t k0, int64_t e, int stride,
                                           const LccTable &tab, uint64_t &cover, int *cnt,
                                           const uint64_t *bits = nullptr) {
    // Blocks of kUnroll entries; the last block is predicated (indices
    // clamped to the last entry, results of out-of-range slots zeroed), so
    // every load of a block is issued before the first wait.
    for (int64_t k = k0; k < e; k += (int64_t)kUnroll * stride) {
        int32_t c[kUnroll];
        bool in[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t kk = k + (int64_t)u * stride;
            in[u] = kk < e;
            c[u] = __builtin_nontemporal_load(col + (in[u] ? kk : e - 1));
        }
        uint64_t x[kUnroll];
        if constexpr (FILT) {
            // all bitmap words first, then all role gathers (inactive
            // neighbours read vertex 0's mask, a shared cached line, and
            // are zeroed): no load waits on a branch
            uint64_t wd[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) wd[u] = bits[c[u] >> 6];
            bool act[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) act[u] = in[u] && ((wd[u] >> (c[u] & 63)) & 1ull);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) x[u] = (uint64_t)omega[act[u] ? c[u] : 0];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) x[u] = act[u] ? x[u] : 0ull;
        } else {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) x[u] = (uint64_t)omega[c[u]];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) x[u] = in[u] ? x[u] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            cover |= x[u];
            if constexpr (CNT) {
#pragma unroll
                for (int q = 0; q < kMaxCount; ++q)
                    if (q < tab.ncount) cnt[q] += (x[u] & tab.cmask[q]) != 0ull;
            }
        }
    }
}

// ------------------------------------------------------- role initialisation
// omega0(v) = { q : l(q) = l(v) } (vertex state and initialisation algorithm)
template <typename M>
__global__ __launch_bounds__(kBlock) void init_roles_kernel(int64_t n, const void *labels,
                                                            int label_bytes, const uint64_t *lut,
                                                            int64_t lut_len, M *omega,
                                                            uint64_t *bits) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t w = 0;
    if (v < n) {
        const int64_t L = label_bytes == 1 ? (int64_t)((const uint8_t *)labels)[v]
                                           : (int64_t)((const uint16_t *)labels)[v];
        w = L < lut_len ? lut[L] : 0ull;
        omega[v] = (M)w;
    }
    // a wavefront covers 64 consecutive vertices: one bitmap word
    const uint64_t m = ballot64(w != 0ull);
    if (bits && lane_id() == 0 && v < n) bits[v >> 6] = m;
}

template <typename M>
void launch_init_roles(hipStream_t s, int64_t n, const void *labels, int label_bytes,
                       const uint64_t *lut, int64_t lut_len, M *omega, uint64_t *bits) {
    if (n <= 0) return;
    int64_t grid = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(init_roles_kernel<M>, dim3((unsigned)grid), dim3(kBlock), 0, s, n, labels,
                       label_bytes, lut, lut_len, omega, bits);
}

// ---------------------------------------------------------------- binning
// The sweep's change flag: set once (a read served by the cache first, so
// that a sweep in which most wavefronts change something does not queue
// thousands of atomics on one address).
__device__ __forceinline__ void mark_changed(int32_t *changed) {
    if (__atomic_load_n(changed, __ATOMIC_RELAXED) == 0) atomicExch(changed, 1);
}

// Bins: 4 lanes per vertex up to wl.bin_small entries, 16 up to
// wl.bin_mid, a wavefront up to kBinWaveMaxDeg, hub segments above (every
// group kernel loops over its row, so the first two bounds are free
// settings; the last is fixed by the hub segmentation).
__device__ __forceinline__ int degree_bin(int64_t d, const Worklists &wl) {
    return d <= wl.bin_small ? 0 : d <= wl.bin_mid ? 1 : d <= kBinWaveMaxDeg ? 2 : 3;
}

// Appends are staged in LDS: a block gathers the selected vertices of a
// chunk of kStageChunk inputs per list with LDS atomics, then reserves space
// in each global list with one atomic and copies the chunk out (one global
// atomic per list per chunk instead of one per wavefront: on graphs with
// tens of millions of vertices the per-wavefront counter atomics serialise).
constexpr int kStageChunk = 2048;
constexpr int kStageRounds = kStageChunk / kBlock;   // entries per thread and chunk

__device__ __forceinline__ void stage_append(bool pred, int32_t v, int32_t *buf, int32_t *cnt) {
    const uint64_t m = ballot64(pred);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt, __popcll(m));
    base = __shfl(base, leader);
    if (pred) buf[base + __popcll(m & lanemask_lt())] = v;
}

template <typename M>
__global__ __launch_bounds__(kBlock) void bin_kernel(const int32_t *in, int64_t n_in,
                                                     const int64_t *rp, const M *omega,
                                                     Worklists wl) {
    __shared__ int32_t buf[kNumBins][kStageChunk];
    __shared__ int32_t cnt[kNumBins], base[kNumBins];
    __shared__ unsigned long long ent;
    for (int64_t c0 = (int64_t)blockIdx.x * kStageChunk; c0 < n_in;
         c0 += (int64_t)gridDim.x * kStageChunk) {
        if (threadIdx.x < kNumBins) cnt[threadIdx.x] = 0;
        if (threadIdx.x == 0) ent = 0;
        __syncthreads();
        unsigned long long tot = 0;
        // every round's loads issued before the first append: one latency
        // per chain of dependent loads instead of one per round
        int32_t vs[kStageRounds];
        bool act[kStageRounds];
        int64_t d[kStageRounds];
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) {
            const int64_t i = c0 + (int64_t)r * kBlock + threadIdx.x;
            act[r] = i < n_in;
            vs[r] = act[r] ? (in ? in[i] : (int32_t)i) : 0;
        }
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) act[r] = act[r] && omega[vs[r]] != 0;
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) d[r] = act[r] ? rp[vs[r] + 1] - rp[vs[r]] : 0;
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) {
            const int b = act[r] ? degree_bin(d[r], wl) : -1;
            tot += (unsigned long long)d[r];
#pragma unroll
            for (int k = 0; k < kNumBins; ++k) stage_append(b == k, vs[r], buf[k], &cnt[k]);
        }
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
        if (lane_id() == 0 && tot) atomicAdd(&ent, tot);
        __syncthreads();
        if (threadIdx.x < kNumBins)
            base[threadIdx.x] =
                cnt[threadIdx.x] ? atomicAdd(wl.count + threadIdx.x, cnt[threadIdx.x]) : 0;
        if (threadIdx.x == 0 && ent) atomicAdd(wl.entries, ent);
        __syncthreads();
        for (int k = 0; k < kNumBins; ++k)
            for (int j = threadIdx.x; j < cnt[k]; j += kBlock) wl.list[k][base[k] + j] = buf[k][j];
        __syncthreads();
    }
}

// Active list: the vertices of `in` (or 0..n-1) whose role set is not empty.
// A block stages kCollectChunk entries in LDS (in groups of kStageRounds
// per thread, each group's loads issued before its appends) and reserves
// their place in the list with one global atomic: the counter is a single
// address, so a pass over all n vertices of a large graph was bound by the
// serialised atomics of 2,048-entry chunks.
constexpr int kCollectChunk = 4 * kStageChunk;
template <typename M>
__global__ __launch_bounds__(kBlock) void collect_kernel(const int32_t *in, int64_t n_in,
                                                         const M *omega, int32_t *out,
                                                         int32_t *counter) {
    __shared__ int32_t buf[kCollectChunk];
    __shared__ int32_t cnt, base;
    for (int64_t c0 = (int64_t)blockIdx.x * kCollectChunk; c0 < n_in;
         c0 += (int64_t)gridDim.x * kCollectChunk) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        for (int g = 0; g < kCollectChunk; g += kStageChunk) {
            int32_t vs[kStageRounds];
            bool live[kStageRounds];
#pragma unroll
            for (int r = 0; r < kStageRounds; ++r) {
                const int64_t i = c0 + g + (int64_t)r * kBlock + threadIdx.x;
                live[r] = i < n_in;
                vs[r] = live[r] ? (in ? in[i] : (int32_t)i) : 0;
            }
#pragma unroll
            for (int r = 0; r < kStageRounds; ++r) live[r] = live[r] && omega[vs[r]] != 0;
#pragma unroll
            for (int r = 0; r < kStageRounds; ++r) stage_append(live[r], vs[r], buf, &cnt);
        }
        __syncthreads();
        if (threadIdx.x == 0) base = cnt ? atomicAdd(counter, cnt) : 0;
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += kBlock) out[base + j] = buf[j];
        __syncthreads();
    }
}

static unsigned stage_grid(int64_t n_in) {
    int64_t g = (n_in + kStageChunk - 1) / kStageChunk;
    return (unsigned)(g > 16384 ? 16384 : g);
}

// ---------------------------------------- first LCC sweep from label counts
// The first LCC sweep evaluated from the initial role sets alone: with
// omega0(u) = roles of u's label, a neighbour u covers template neighbour
// q' of q iff label(u) = label(q'), and the distinct-count rule for label L
// counts exactly the neighbours of label L.  So role q of v survives the
// first sweep iff, for every label L, v has at least need_q(L) neighbours
// of label L (need_q(L) = template neighbours of q with label L).  This is
// the first Jacobi iteration of the LCC rule; later sweeps continue from
// it to the same greatest fixpoint.  Each thread takes 4 consecutive
// vertices: one 4-byte label load, one 4-byte load per needed label column
// (all independent), and writes omega for every vertex (this also
// initialises it).
template <typename M>
__global__ __launch_bounds__(kBlock) void first_sweep_counts_kernel(
    int64_t n, int64_t np, const uint8_t *labels, const uint64_t *lut, int lut_len,
    const uint8_t *cnt, int nlab, const int32_t *need_off, const int32_t *need_lab,
    const int32_t *need_min, int n0, M *omega, bool aligned) {
    __shared__ uint64_t s_lut[256];
    __shared__ uint8_t s_need[kMaxK][kCountLabels];   // need_q(L), 0 if none
    __shared__ uint64_t s_lmask[kMaxK];               // labels q needs
    __shared__ int32_t s_drop[kMaxK];                 // q needs a label with no column
    for (int i = threadIdx.x; i < lut_len; i += blockDim.x) s_lut[i] = lut[i];
    for (int q = threadIdx.x; q < n0; q += blockDim.x) {
        for (int L = 0; L < kCountLabels; ++L) s_need[q][L] = 0;
        uint64_t lm = 0;
        int drop = 0;
        for (int i = need_off[q]; i < need_off[q + 1]; ++i) {
            const int L = need_lab[i];
            if (L < nlab) {
                s_need[q][L] = (uint8_t)(need_min[i] > 255 ? 255 : need_min[i]);
                lm |= 1ull << L;
            } else {
                drop = 1;
            }
        }
        s_lmask[q] = lm;
        s_drop[q] = drop;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t v4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; v4 < n; v4 += stride) {
        const bool full = aligned && v4 + 4 <= n;
        uint32_t lab4;
        if (full) {
            lab4 = *reinterpret_cast<const uint32_t *>(labels + v4);
        } else {
            lab4 = 0;
            for (int i = 0; i < 4 && v4 + i < n; ++i) lab4 |= (uint32_t)labels[v4 + i] << (8 * i);
        }
        uint64_t w[4];
        uint64_t need = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int lab = (int)((lab4 >> (8 * i)) & 0xffu);
            w[i] = (v4 + i < n && lab < lut_len) ? s_lut[lab] : 0ull;
            for (uint64_t b = w[i]; b; b &= b - 1) {
                const int q = __builtin_ctzll(b);
                if (s_drop[q]) w[i] &= ~(1ull << q);
                need |= s_lmask[q];
            }
        }
        for (uint64_t lb = need; lb; lb &= lb - 1) {
            const int L = __builtin_ctzll(lb);
            const uint32_t c4 = *reinterpret_cast<const uint32_t *>(cnt + (int64_t)L * np + v4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t c = (c4 >> (8 * i)) & 0xffu;
                for (uint64_t b = w[i]; b; b &= b - 1) {
                    const int q = __builtin_ctzll(b);
                    if (c < s_need[q][L]) w[i] &= ~(1ull << q);
                }
            }
        }
        if (full && sizeof(M) == 1) {
            const uint32_t o = (uint32_t)w[0] | ((uint32_t)w[1] << 8) | ((uint32_t)w[2] << 16) |
                               ((uint32_t)w[3] << 24);
            *reinterpret_cast<uint32_t *>(omega + v4) = o;
        } else {
            for (int i = 0; i < 4; ++i)
                if (v4 + i < n) omega[v4 + i] = (M)w[i];
        }
    }
}

template <typename M>
void launch_first_sweep_counts(hipStream_t s, int64_t n, int64_t np, const uint8_t *labels,
                               const uint64_t *lut, int lut_len, const uint8_t *cnt, int nlab,
                               const int32_t *need_off, const int32_t *need_lab,
                               const int32_t *need_min, int n0, M *omega) {
    if (n <= 0) return;
    int64_t grid = ((n + 3) / 4 + kBlock - 1) / kBlock;
    if (grid > (1 << 20)) grid = 1 << 20;
    // 4-byte label loads and omega stores need 4-byte aligned arrays (a
    // borrowed label tensor may start anywhere)
    const bool aligned = ((uintptr_t)labels % 4 == 0) && ((uintptr_t)omega % 4 == 0);
    hipLaunchKernelGGL(first_sweep_counts_kernel<M>, dim3((unsigned)grid), dim3(kBlock), 0, s, n,
                       np, labels, lut, lut_len, cnt, nlab, need_off, need_lab, need_min, n0,
                       omega, aligned);
}

template <typename M>
void launch_collect(hipStream_t s, const int32_t *in, int64_t n_in, const M *omega,
                    int32_t *out, int32_t *counter) {
    if (n_in <= 0) return;
    int64_t g = (n_in + kCollectChunk - 1) / kCollectChunk;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(collect_kernel<M>, dim3((unsigned)g), dim3(kBlock), 0, s, in, n_in, omega,
                       out, counter);
}

template <typename M>
void launch_bin(hipStream_t s, const int32_t *in, int64_t n_in, const int64_t *rp,
                const M *omega, Worklists &wl) {
    if (n_in <= 0) return;
    hipLaunchKernelGGL(bin_kernel<M>, dim3(stage_grid(n_in)), dim3(kBlock), 0, s, in, n_in, rp,
                       omega, wl);
}

// Hub vertices are split into segments of kHubSegment entries, one wavefront
// each; a single block assigns segments with a block-wide exclusive scan.
// Hub segments: one thread per hub vertex takes a contiguous range of
// segment slots from the shared counter *n_seg (zeroed by the caller) and
// writes its segments in row order; hubs may take their ranges in any order
// (consumers only need each hub's segments contiguous and ascending).
// Slots and per-hub records beyond the capacities are not written, but
// *n_seg still counts every segment so the host can detect the overflow.
__global__ __launch_bounds__(kBlock) void hub_segments_kernel(const int64_t *__restrict__ rp,
                                                              Worklists wl) {
    const int64_t n_hubs = wl.count[3];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_hubs;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = wl.list[3][i];
        const int64_t b = rp[v];
        const int64_t d = rp[v + 1] - b;
        const int64_t ns = (d + kHubSegment - 1) / kHubSegment;
        const int64_t first = atomicAdd(wl.n_seg, (int32_t)ns);
        if (i >= wl.hub_capacity) continue;
        for (int64_t k = 0; k < ns; ++k) {
            const int64_t seg = first + k;
            if (seg >= wl.seg_capacity) break;
            wl.hub_seg_v[seg] = v;
            wl.hub_seg_begin[seg] = b + k * kHubSegment;
            wl.hub_seg_end[seg] = (k + 1) * kHubSegment < d ? b + (k + 1) * kHubSegment : b + d;
            wl.hub_seg_slot[seg] = (int32_t)i;
        }
        wl.hub_nseg[i] = (int32_t)ns;
        wl.hub_seg_first[i] = (int32_t)first;
        wl.hub_cover[i] = 0;
        wl.hub_ticket[i] = 0;
        for (int c = 0; c < kMaxCount; ++c) wl.hub_count[i * kMaxCount + c] = 0;
    }
}

void launch_hub_segments(hipStream_t s, const int64_t *rp, Worklists &wl, int64_t) {
    hipLaunchKernelGGL(hub_segments_kernel, dim3(256), dim3(kBlock), 0, s, rp, wl);
}

// ------------------------------------------------------------- LCC sweep
// One launch per sweep.  Blocks are assigned to degree bins by blockIdx
// ranges: G = 4, 16 or 64 lanes per vertex for the three lower bins, one
// wavefront per segment of kHubSegment entries for the hub bin, whose
// partial coverage and counts are combined with atomics; the last segment
// of a vertex (ticket) applies the rule.
template <typename M, int G, bool CNT, bool FILT>
__device__ __forceinline__ void lcc_group_body(int64_t local_block, const int64_t *__restrict__ rp,
                                               const int32_t *__restrict__ col, M *omega,
                                               const int32_t *__restrict__ list, int64_t count,
                                               const LccTable &tab, int32_t *changed,
                                               const uint64_t *bits) {
    const int lane = lane_id();
    const int sl = lane & (G - 1);
    const int64_t idx = (local_block * blockDim.x + threadIdx.x) / G;
    const bool valid = idx < count;
    const int32_t v = valid ? list[idx] : 0;
    const uint64_t w = valid ? (uint64_t)omega[v] : 0ull;
    int64_t s = 0, e = 0;
    if (w) {
        s = rp[v];
        e = rp[v + 1];
    }
    uint64_t cover = 0;
    int cnt[CNT ? kMaxCount : 1];
#pragma unroll
    for (int c = 0; c < (CNT ? kMaxCount : 1); ++c) cnt[c] = 0;
    accumulate<M, CNT, FILT>(col, omega, s + sl, e, G, tab, cover, cnt, bits);
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        cover |= shfl_xor_u64(cover, off, G);
        if constexpr (CNT) {
#pragma unroll
            for (int c = 0; c < kMaxCount; ++c)
                if (c < tab.ncount) cnt[c] += __shfl_xor(cnt[c], off, G);
        }
    }
    bool ch = false;
    if (w && sl == 0) {
        uint64_t nw = evaluate<CNT>(w, cover, cnt, tab);
        if (nw != w) {
            omega[v] = (M)nw;
            ch = true;
        }
    }
    if (ballot64(ch) && lane == 0) mark_changed(changed);
}

template <typename M, bool CNT, bool FILT>
__device__ __forceinline__ void lcc_hub_body(int64_t local_block, const int64_t *__restrict__ rp,
                                             const int32_t *__restrict__ col, M *omega,
                                             const Worklists &wl, int64_t n_seg,
                                             const LccTable &tab, int32_t *changed,
                                             const uint64_t *bits) {
    const int lane = lane_id();
    const int64_t seg = (local_block * blockDim.x + threadIdx.x) / kWave;
    if (seg >= n_seg) return;
    const int32_t v = wl.hub_seg_v[seg];
    const int32_t slot = wl.hub_seg_slot[seg];
    const int64_t b = wl.hub_seg_begin[seg], e = wl.hub_seg_end[seg];
    uint64_t cover = 0;
    int cnt[CNT ? kMaxCount : 1];
#pragma unroll
    for (int c = 0; c < (CNT ? kMaxCount : 1); ++c) cnt[c] = 0;
    accumulate<M, CNT, FILT>(col, omega, b + lane, e, kWave, tab, cover, cnt, bits);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cover |= shfl_xor_u64(cover, off, 64);
        if constexpr (CNT) {
#pragma unroll
            for (int c = 0; c < kMaxCount; ++c)
                if (c < tab.ncount) cnt[c] += __shfl_xor(cnt[c], off, 64);
        }
    }
    if (lane == 0) {
        atomicOr((unsigned long long *)&wl.hub_cover[slot], (unsigned long long)cover);
        if constexpr (CNT) {
            for (int c = 0; c < tab.ncount; ++c)
                atomicAdd(&wl.hub_count[slot * kMaxCount + c], cnt[c]);
        }
        __threadfence();
        int t = atomicAdd(&wl.hub_ticket[slot], 1);
        if (t == wl.hub_nseg[slot] - 1) {
            __threadfence();
            uint64_t cov = atomicOr((unsigned long long *)&wl.hub_cover[slot], 0ull);
            int tot[CNT ? kMaxCount : 1];
            if constexpr (CNT) {
#pragma unroll
                for (int c = 0; c < kMaxCount; ++c)
                    tot[c] = c < tab.ncount ? atomicAdd(&wl.hub_count[slot * kMaxCount + c], 0) : 0;
            }
            const uint64_t w = (uint64_t)omega[v];
            const uint64_t nw = evaluate<CNT>(w, cov, tot, tab);
            wl.hub_cover[slot] = 0;
            wl.hub_ticket[slot] = 0;
            if constexpr (CNT) {
                for (int c = 0; c < tab.ncount; ++c) wl.hub_count[slot * kMaxCount + c] = 0;
            }
            if (nw != w) {
                omega[v] = (M)nw;
                mark_changed(changed);
            }
        }
    }
}

struct SweepGrid {
    int64_t count[3];        // vertices in bins 0..2
    int64_t n_seg;           // hub segments
    int64_t start[5];        // first block of each bin; start[4] = total blocks
};

static SweepGrid sweep_grid(const int64_t *hc, int64_t n_seg) {
    SweepGrid g{};
    const int per[4] = {kBlock / 4, kBlock / 16, kBlock / 64, kBlock / 64};
    int64_t items[4] = {hc[0], hc[1], hc[2], n_seg};
    g.start[0] = 0;
    for (int b = 0; b < 4; ++b) g.start[b + 1] = g.start[b] + (items[b] + per[b] - 1) / per[b];
    for (int b = 0; b < 3; ++b) g.count[b] = hc[b];
    g.n_seg = n_seg;
    return g;
}

// FULL distinguishes the first sweep over the whole graph (its own kernel
// symbol, so that profiles report it separately) from the sweeps over the
// compacted candidate subgraph.
template <typename M, bool CNT, bool FULL>
__global__ __launch_bounds__(kBlock) void lcc_sweep_kernel(const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           M *omega, Worklists wl, SweepGrid sg,
                                                           LccTable tab, int32_t *changed,
                                                           const uint64_t *bits) {
    const int64_t b = blockIdx.x;
    if (b < sg.start[1])
        lcc_group_body<M, 4, CNT, FULL>(b, rp, col, omega, wl.list[0], sg.count[0], tab, changed,
                                        bits);
    else if (b < sg.start[2])
        lcc_group_body<M, 16, CNT, FULL>(b - sg.start[1], rp, col, omega, wl.list[1], sg.count[1],
                                         tab, changed, bits);
    else if (b < sg.start[3])
        lcc_group_body<M, 64, CNT, FULL>(b - sg.start[2], rp, col, omega, wl.list[2], sg.count[2],
                                         tab, changed, bits);
    else
        lcc_hub_body<M, CNT, FULL>(b - sg.start[3], rp, col, omega, wl, sg.n_seg, tab, changed,
                                   bits);
}

template <typename M, bool CNT>
static void sweep_impl(hipStream_t s, const int64_t *rp, const int32_t *col, M *omega,
                       const Worklists &wl, const int64_t *hc, int64_t n_seg,
                       const LccTable &tab, int32_t *changed, bool full) {
    SweepGrid sg = sweep_grid(hc, n_seg);
    if (sg.start[4] == 0) return;
    if (full)
        hipLaunchKernelGGL((lcc_sweep_kernel<M, CNT, true>), dim3((unsigned)sg.start[4]),
                           dim3(kBlock), 0, s, rp, col, omega, wl, sg, tab, changed, wl.act_bits);
    else
        hipLaunchKernelGGL((lcc_sweep_kernel<M, CNT, false>), dim3((unsigned)sg.start[4]),
                           dim3(kBlock), 0, s, rp, col, omega, wl, sg, tab, changed, nullptr);
}

template <typename M>
void launch_lcc_sweep(hipStream_t s, const int64_t *rp, const int32_t *col, M *omega,
                      const Worklists &wl, const int64_t *host_counts, int64_t n_seg,
                      const LccTable &tab, int32_t *changed, bool full) {
    if (tab.ncount > 0)
        sweep_impl<M, true>(s, rp, col, omega, wl, host_counts, n_seg, tab, changed, full);
    else
        sweep_impl<M, false>(s, rp, col, omega, wl, host_counts, n_seg, tab, changed, full);
}

// ---------------------------------------------------- subgraph compaction
// Entry u->w is kept iff omega(w) meets the roles adjacent to omega(u): the
// edge elimination of the LCC description (edges to eliminated neighbours
// and to neighbours of non-adjacent roles are dropped).
// Coarse filter of the vertices active when it was built: bit g of the
// filter is set iff one of the vertices 8g .. 8g+7 had a role then.  Role
// sets only shrink during a prune, so a clear bit proves omega[x] == 0 and
// the compaction skips the gather of omega[x]; one bit per eight vertices
// keeps the filter small enough (n/64 bytes) to stay in L2 while the role
// sets of a large graph do not.  A null filter passes every vertex.
constexpr int kFiltShift = 3;
__device__ __forceinline__ bool may_be_active(const uint32_t *__restrict__ f, int32_t x) {
    return !f || ((f[x >> (kFiltShift + 5)] >> ((x >> kFiltShift) & 31)) & 1u);
}
template <typename M>
__device__ __forceinline__ uint64_t omega_filtered(const M *__restrict__ omega,
                                                   const uint32_t *__restrict__ f, int32_t x) {
    return may_be_active(f, x) ? (uint64_t)omega[x] : 0ull;
}

// Is entry u -> x kept (reach: the roles adjacent to omega(u))?  With the
// edge elimination ablated every entry of an active row is kept.
template <typename M>
__device__ __forceinline__ bool keeps(const M *__restrict__ omega,
                                      const uint32_t *__restrict__ f, int32_t x, uint64_t reach,
                                      const LccTable &tab) {
    return tab.keep_all || (omega_filtered(omega, f, x) & reach) != 0ull;
}

// One thread per vertex over ceil(n / 256) * 256 threads: a wavefront's
// ballot of non-empty role sets (64 vertices) folds to 8 filter bits, one
// byte of the filter, so every byte is written and no clearing is needed.
template <typename M>
__global__ __launch_bounds__(kBlock) void active_filter_kernel(int64_t n, const M *omega,
                                                               uint8_t *filt) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t b = ballot64(v < n && omega[v] != 0);
    if (lane_id() == 0) {
        uint32_t byte = 0;
        for (int g = 0; g < 8; ++g)
            if ((b >> (8 * g)) & 0xFFull) byte |= 1u << g;
        filt[v >> 6] = (uint8_t)byte;
    }
}

template <typename M>
void launch_active_filter(hipStream_t s, int64_t n, const M *omega, uint32_t *filt) {
    const int64_t words = (n + 255) / 256;
    if (words <= 0) return;
    hipLaunchKernelGGL(active_filter_kernel<M>, dim3((unsigned)words), dim3(kBlock), 0, s, n,
                       omega, reinterpret_cast<uint8_t *>(filt));
}

template <typename M, int G>
__global__ __launch_bounds__(kBlock) void compact_count_group(const int64_t *__restrict__ rp,
                                                              const int32_t *__restrict__ col,
                                                              const M *__restrict__ omega,
                                                              const int32_t *__restrict__ list,
                                                              int64_t count, LccTable tab,
                                                              const uint32_t *__restrict__ filt,
                                                              int32_t *deg_out) {
    const int sl = lane_id() & (G - 1);
    const int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const bool valid = idx < count;
    const int32_t v = valid ? list[idx] : 0;
    const uint64_t w = valid ? (uint64_t)omega[v] : 0ull;
    const uint64_t reach = reach_of<M>(w, tab);
    int64_t s = 0, e = 0;
    if (reach) {
        s = rp[v];
        e = rp[v + 1];
    }
    int c = 0;
    {
        int64_t k = s + sl;
        for (; k + (int64_t)(kUnroll - 1) * G < e; k += (int64_t)kUnroll * G) {
            int32_t cc[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) cc[u] = col[k + (int64_t)u * G];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                c += keeps(omega, filt, cc[u], reach, tab);
        }
        for (; k < e; k += G) c += keeps(omega, filt, col[k], reach, tab);
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, G);
    if (valid && sl == 0) deg_out[v] = c;
}

// Hub segments (kHubSegment entries, one wavefront each): the count pass
// stores the keep ballot of every 64-entry chunk (seg_bits, 64 words per
// segment), so the fill pass reads the columns of kept entries only and
// gathers no role sets.
template <typename M>
__global__ __launch_bounds__(kBlock) void compact_count_hub(const int64_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const M *__restrict__ omega,
                                                            Worklists wl, int64_t n_seg,
                                                            LccTable tab,
                                                            const uint32_t *__restrict__ filt,
                                                            int32_t *deg_out,
                                                            int64_t *seg_count,
                                                            uint64_t *seg_bits) {
    const int lane = lane_id();
    const int64_t seg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (seg >= n_seg) return;
    const int32_t v = wl.hub_seg_v[seg];
    const uint64_t reach = reach_of<M>((uint64_t)omega[v], tab);
    int64_t c = 0;
    if (reach) {
        const int64_t b = wl.hub_seg_begin[seg], e = wl.hub_seg_end[seg];
        uint64_t *bits = seg_bits + seg * (kHubSegment / kWave);
        int chunk = 0;
        int64_t k0 = b;
        for (; k0 + (int64_t)kUnroll * kWave <= e; k0 += (int64_t)kUnroll * kWave) {
            int32_t cc[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) cc[u] = col[k0 + (int64_t)u * kWave + lane];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t m = ballot64(keeps(omega, filt, cc[u], reach, tab));
                if (lane == 0) bits[chunk + u] = m;
                c += __popcll(m);
            }
            chunk += kUnroll;
        }
        for (; k0 < e; k0 += kWave, ++chunk) {
            const int64_t k = k0 + lane;
            const uint64_t m =
                ballot64(k < e && keeps(omega, filt, col[k], reach, tab));
            if (lane == 0) bits[chunk] = m;
            c += __popcll(m);
        }
    }
    if (lane == 0) {
        seg_count[seg] = c;
        if (c) atomicAdd(&deg_out[v], (int32_t)c);
    }
}

template <typename M, int G>
__global__ __launch_bounds__(kBlock) void compact_fill_group(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ col, const M *__restrict__ omega,
    const int32_t *__restrict__ list, int64_t count, LccTable tab, const uint32_t *__restrict__ filt,
    const int64_t *__restrict__ c_rp, const int32_t *__restrict__ base_off, int32_t *c_col,
    int32_t *c_off, int32_t *c_own) {
    const int lane = lane_id();
    const int sl = lane & (G - 1);
    const int sub_shift = lane & ~(G - 1);
    const int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const bool valid = idx < count;
    const int32_t v = valid ? list[idx] : 0;
    const uint64_t w = valid ? (uint64_t)omega[v] : 0ull;
    const uint64_t reach = reach_of<M>(w, tab);
    int64_t s = 0, e = 0, pos = 0;
    if (reach) {
        s = rp[v];
        e = rp[v + 1];
        pos = c_rp[v];
    }
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << sub_shift);
    // every lane of the wavefront runs the same number of iterations so the
    // ballots stay convergent
    int64_t my_iters = (e - s + G - 1) / G;
    int64_t iters = my_iters;
    for (int off = 32; off > 0; off >>= 1) {
        int64_t o = __shfl_xor(iters, off, 64);
        iters = o > iters ? o : iters;
    }
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t k = s + it * G + sl;
        bool keep = false;
        int32_t x = 0;
        if (k < e) {
            x = col[k];
            keep = keeps(omega, filt, x, reach, tab);
        }
        const uint64_t m = ballot64(keep) & gmask;
        if (keep) {
            const int64_t p = pos + __popcll(m & lanemask_lt());
            c_col[p] = x;
            c_off[p] = base_off ? base_off[k] : (int32_t)(k - s);
            c_own[p] = v;
        }
        pos += __popcll(m);
    }
}

template <typename M>
__global__ __launch_bounds__(kBlock) void compact_fill_hub(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ col, const M *__restrict__ omega,
    Worklists wl, int64_t n_seg, LccTable tab, const int64_t *__restrict__ c_rp,
    const int64_t *__restrict__ seg_scan, const uint64_t *__restrict__ seg_bits,
    const int32_t *__restrict__ base_off, int32_t *__restrict__ c_col,
    int32_t *__restrict__ c_off, int32_t *__restrict__ c_own) {
    const int lane = lane_id();
    const int64_t seg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (seg >= n_seg) return;
    const int32_t v = wl.hub_seg_v[seg];
    const int32_t slot = wl.hub_seg_slot[seg];
    const uint64_t reach = reach_of<M>((uint64_t)omega[v], tab);
    if (!reach) return;
    // offset of this segment in v's compacted row: kept entries of the
    // slot's earlier segments (exclusive scan over all segments)
    const int64_t pos = c_rp[v] + seg_scan[seg] - seg_scan[wl.hub_seg_first[slot]];
    const int64_t row0 = rp[v];
    const int64_t b = wl.hub_seg_begin[seg], e = wl.hub_seg_end[seg];
    // lane c holds the keep ballot of chunk c (at most 64 chunks per
    // segment) and the number of kept entries of the chunks before it, so
    // the chunks are independent: no chain of dependent loads
    const int nchunks = (int)((e - b + kWave - 1) / kWave);
    const uint64_t mine = lane < nchunks ? seg_bits[seg * (kHubSegment / kWave) + lane] : 0ull;
    int32_t before = __popcll(mine);
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t t = __shfl_up(before, off, kWave);
        if (lane >= off) before += t;
    }
    before -= __popcll(mine);
    for (uint64_t live = ballot64(mine != 0ull); live; live &= live - 1) {
        const int chunk = __builtin_ctzll(live);
        const uint64_t m = read_lane_u64(mine, chunk);
        if ((m >> lane) & 1ull) {
            const int64_t k = b + (int64_t)chunk * kWave + lane;
            const int64_t p = pos + read_lane32(before, chunk) + __popcll(m & lanemask_lt());
            c_col[p] = col[k];
            c_off[p] = base_off ? base_off[k] : (int32_t)(k - row0);
            c_own[p] = v;
        }
    }
}

template <typename M>
void launch_compact_count(hipStream_t s, const int64_t *rp, const int32_t *col, const M *omega,
                          const Worklists &wl, const int64_t *hc, int64_t n_seg,
                          const LccTable &tab, const uint32_t *filt, int32_t *deg_out,
                          int64_t *seg_count, uint64_t *seg_bits) {
    if (hc[0] > 0)
        hipLaunchKernelGGL((compact_count_group<M, 4>),
                           dim3((unsigned)((hc[0] * 4 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           rp, col, omega, wl.list[0], hc[0], tab, filt, deg_out);
    if (hc[1] > 0)
        hipLaunchKernelGGL((compact_count_group<M, 16>),
                           dim3((unsigned)((hc[1] * 16 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, rp, col, omega, wl.list[1], hc[1], tab, filt, deg_out);
    if (hc[2] > 0)
        hipLaunchKernelGGL((compact_count_group<M, 64>),
                           dim3((unsigned)((hc[2] * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, rp, col, omega, wl.list[2], hc[2], tab, filt, deg_out);
    if (n_seg > 0)
        hipLaunchKernelGGL((compact_count_hub<M>),
                           dim3((unsigned)((n_seg * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, rp, col, omega, wl, n_seg, tab, filt, deg_out, seg_count, seg_bits);
}

template <typename M>
void launch_compact_fill(hipStream_t s, const int64_t *rp, const int32_t *col, const M *omega,
                         const Worklists &wl, const int64_t *hc, int64_t n_seg,
                         const LccTable &tab, const uint32_t *filt, const int64_t *c_rp,
                         const int64_t *seg_scan, const uint64_t *seg_bits,
                         const int32_t *base_off, int32_t *c_col, int32_t *c_off,
                         int32_t *c_own) {
    if (hc[0] > 0)
        hipLaunchKernelGGL((compact_fill_group<M, 4>),
                           dim3((unsigned)((hc[0] * 4 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           rp, col, omega, wl.list[0], hc[0], tab, filt, c_rp, base_off, c_col, c_off,
                           c_own);
    if (hc[1] > 0)
        hipLaunchKernelGGL((compact_fill_group<M, 16>),
                           dim3((unsigned)((hc[1] * 16 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, rp, col, omega, wl.list[1], hc[1], tab, filt, c_rp, base_off, c_col, c_off,
                           c_own);
    if (hc[2] > 0)
        hipLaunchKernelGGL((compact_fill_group<M, 64>),
                           dim3((unsigned)((hc[2] * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, rp, col, omega, wl.list[2], hc[2], tab, filt, c_rp, base_off, c_col, c_off,
                           c_own);
    if (n_seg > 0)
        hipLaunchKernelGGL((compact_fill_hub<M>),
                           dim3((unsigned)((n_seg * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, rp, col, omega, wl, n_seg, tab, c_rp, seg_scan, seg_bits, base_off,
                           c_col, c_off, c_own);
}

// --------------------------------------------------------- exclusive scan
__global__ void fill_from_kernel(const int64_t *src, int64_t *dst) { *dst = *src; }

// out[i] = in[0] + ... + in[i-1] for i in [0, n]; three passes over tiles of
// kScanTile elements.
constexpr int kScanPer = 16;
constexpr int kScanTile = kBlock * kScanPer;

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_tile_sums(const T *in, int64_t n, int64_t *sums) {
    __shared__ int64_t red[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int j = 0; j < kScanPer; ++j) {
        int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < n) acc += (int64_t)in[i];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane_id() == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
        sums[blockIdx.x] = t;
    }
}

// Block-wide exclusive scan of one value per thread (kBlock threads): wave
// scans by shuffles, then the wave totals through LDS.  Returns the
// exclusive prefix; *total receives the block's sum.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t *wsum,
                                                        int64_t *total) {
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    int64_t inc = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t t = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += t;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        const int64_t v = wsum[i];
        if (i < w) before += v;
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

// One tile of kScanTile elements, coalesced: staged through LDS (rows of
// kScanPer elements padded by one, so a thread's row reads hit distinct
// banks), each thread sums its row, the block scans the row sums, and the
// exclusive prefixes go back through LDS to coalesced stores.  in may equal
// out (64-bit input).  base_add is added to every output.
template <typename T>
__device__ __forceinline__ void scan_tile(const T *in, int64_t *out, int64_t n,
                                          int64_t tile0, int64_t base_add, int64_t *stage,
                                          int64_t *wsum, int64_t *tile_total) {
    constexpr int kPad = kScanPer + 1;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int e = j * kBlock + threadIdx.x;          // element within the tile
        const int64_t i = tile0 + e;
        stage[(e / kScanPer) * kPad + (e % kScanPer)] = i < n ? (int64_t)in[i] : 0;
    }
    __syncthreads();
    int64_t row = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) row += stage[threadIdx.x * kPad + j];
    int64_t total = 0;
    int64_t run = block_exclusive_scan(row, wsum, &total) + base_add;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t v = stage[threadIdx.x * kPad + j];
        stage[threadIdx.x * kPad + j] = run;
        run += v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int e = j * kBlock + threadIdx.x;
        const int64_t i = tile0 + e;
        if (i < n) out[i] = stage[(e / kScanPer) * kPad + (e % kScanPer)];
    }
    __syncthreads();
    *tile_total = total;
}

// Exclusive scan of at most kScanTile values in place; *total_out receives
// their sum.
__global__ __launch_bounds__(kBlock) void scan_small_kernel(int64_t *a, int64_t n,
                                                            int64_t *total_out) {
    __shared__ int64_t stage[kBlock * (kScanPer + 1)];
    __shared__ int64_t wsum[kBlock / kWave];
    int64_t total = 0;
    scan_tile<int64_t>(a, a, n, 0, 0, stage, wsum, &total);
    if (threadIdx.x == 0) *total_out = total;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_apply(const T *in, int64_t n, const int64_t *sums,
                                                     int64_t *out) {
    __shared__ int64_t stage[kBlock * (kScanPer + 1)];
    __shared__ int64_t wsum[kBlock / kWave];
    int64_t total = 0;
    scan_tile<T>(in, out, n, (int64_t)blockIdx.x * kScanTile, sums[blockIdx.x], stage, wsum,
                 &total);
}

// Tile sums, an exclusive scan of the tile sums (in one block when there
// are at most kScanTile of them, else recursively), then every tile scanned
// with its offset.  scratch holds scan_scratch_len(n) values.  T: int64_t
// or int32_t input (the output is 64-bit either way).
template <typename T>
void launch_exclusive_scan(hipStream_t s, const T *in, int64_t *out, int64_t n, int64_t *scratch,
                           int64_t len) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(scan_tile_sums<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, scratch);
    if (nb <= kScanTile) {
        hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(kBlock), 0, s, scratch, nb, out + n);
    } else {
        // scratch[0, nb) scanned in place; its total to out[n]
        launch_exclusive_scan<int64_t>(s, scratch, scratch, nb, scratch + nb + 1, len - nb - 1);
        hipLaunchKernelGGL(fill_from_kernel, dim3(1), dim3(1), 0, s, scratch + nb, out + n);
    }
    hipLaunchKernelGGL(scan_apply<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, scratch, out);
}
template void launch_exclusive_scan<int64_t>(hipStream_t, const int64_t *, int64_t *, int64_t,
                                             int64_t *, int64_t);
template void launch_exclusive_scan<int32_t>(hipStream_t, const int32_t *, int64_t *, int64_t,
                                             int64_t *, int64_t);

int64_t scan_scratch_len(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    return nb + 1 + (nb > kScanTile ? scan_scratch_len(nb) : 0);
}

// ---------------------------------------------------------------- fills
__global__ void fill_u64_kernel(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_u64(hipStream_t s, uint64_t *p, int64_t n, uint64_t v) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)g), dim3(kBlock), 0, s, p, n, v);
}
void launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)g), dim3(kBlock), 0, s, p, n, v);
}

__global__ void label_hist_kernel(int64_t n, const void *labels, int label_bytes,
                                  unsigned long long *hist, int64_t hist_len) {
    // 8-bit labels: per-block histogram in LDS, one global atomic per bin
    __shared__ unsigned int local[256];
    const bool small = label_bytes == 1 && hist_len <= 256;
    if (small) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) local[i] = 0;
        __syncthreads();
    }
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t L = label_bytes == 1 ? (int64_t)((const uint8_t *)labels)[v]
                                     : (int64_t)((const uint16_t *)labels)[v];
        if (L < hist_len) {
            if (small) atomicAdd(&local[L], 1u);
            else atomicAdd(&hist[L], 1ull);
        }
    }
    if (small) {
        __syncthreads();
        for (int i = threadIdx.x; i < 256; i += blockDim.x)
            if (local[i]) atomicAdd(&hist[i], (unsigned long long)local[i]);
    }
}

void launch_label_hist(hipStream_t s, int64_t n, const void *labels, int label_bytes,
                       unsigned long long *hist, int64_t hist_len) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(label_hist_kernel, dim3((unsigned)g), dim3(kBlock), 0, s, n, labels,
                       label_bytes, hist, hist_len);
}

template <typename M>
__global__ void widen_kernel(int64_t n, const M *src, uint64_t *dst) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        dst[v] = (uint64_t)src[v];
}

template <typename M>
void launch_widen(hipStream_t s, int64_t n, const M *src, uint64_t *dst) {
    if (n <= 0) return;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(widen_kernel<M>, dim3((unsigned)g), dim3(kBlock), 0, s, n, src, dst);
}

#define PM_INSTANTIATE_LCC(M)                                                                     \
    template void launch_init_roles<M>(hipStream_t, int64_t, const void *, int, const uint64_t *, \
                                       int64_t, M *, uint64_t *);                                 \
    template void launch_bin<M>(hipStream_t, const int32_t *, int64_t, const int64_t *,            \
                                const M *, Worklists &);                                          \
    template void launch_lcc_sweep<M>(hipStream_t, const int64_t *, const int32_t *, M *,          \
                                      const Worklists &, const int64_t *, int64_t,                \
                                      const LccTable &, int32_t *, bool);                         \
    template void launch_compact_count<M>(hipStream_t, const int64_t *, const int32_t *,           \
                                          const M *, const Worklists &, const int64_t *, int64_t, \
                                          const LccTable &, const uint32_t *, int32_t *,          \
                                          int64_t *, uint64_t *);                                 \
    template void launch_active_filter<M>(hipStream_t, int64_t, const M *, uint32_t *);          \
    template void launch_compact_fill<M>(hipStream_t, const int64_t *, const int32_t *, const M *, \
                                         const Worklists &, const int64_t *, int64_t,             \
                                         const LccTable &, const uint32_t *, const int64_t *,     \
                                         const int64_t *,                                         \
                                         const uint64_t *, const int32_t *, int32_t *, int32_t *,  \
                                         int32_t *);                                              \
    template void launch_widen<M>(hipStream_t, int64_t, const M *, uint64_t *);                  \
    template void launch_collect<M>(hipStream_t, const int32_t *, int64_t, const M *, int32_t *,  \
                                    int32_t *);                                                   \
    template void launch_first_sweep_counts<M>(                                                   \
        hipStream_t, int64_t, int64_t, const uint8_t *, const uint64_t *, int, const uint8_t *,   \
        int, const int32_t *, const int32_t *, const int32_t *, int, M *);

PM_INSTANTIATE_LCC(uint8_t)
PM_INSTANTIATE_LCC(uint16_t)
PM_INSTANTIATE_LCC(uint32_t)
PM_INSTANTIATE_LCC(uint64_t)

}  // namespace pm
