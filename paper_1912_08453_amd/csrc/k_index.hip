// Neighbour-label count index for gfx950: cnt[L * np + v] = number of
// neighbours of v with label L, saturated at 255 (uint8 labels below
// kCountLabels; np = n rounded up to a multiple of 256, the padding holds
// zeros).  With omega0(u) = roles of u's label, the first LCC sweep of every
// template is a function of these counts alone (first_sweep_counts_kernel),
// so this one pass over the CSR serves the first sweep of every template
// pruned on the graph.
//
// The pass streams the CSR once: row_ptr and col are read sequentially, the
// label of every column is gathered (1 byte), and each label's counts are
// written as 256-byte runs.
//  * Tiles: a block owns 256 consecutive vertices, whose rows are one
//    contiguous stretch of col.  All 256 threads stream that stretch in
//    order (entry k of the stretch goes to thread k mod 256), eight entries
//    per thread in flight, so short rows do not leave lanes idle.  An
//    entry's row is found by binary search over the tile's 257 row starts
//    in LDS, and the count goes to a 16-bit LDS counter (two labels per
//    32-bit word, no global atomics).  The block then writes the saturated
//    counts label by label, 4 vertices per 32-bit store.
//  * Hubs: rows longer than kBinWaveMaxDeg are cut out of their tile's
//    stretch and counted by segments of kHubSegment entries, one wavefront
//    each, with per-wavefront LDS counters added into 32-bit global
//    counters per (hub, label); a last kernel saturates those into the index.
#include "device_util.h"
#include "pm_internal.h"

namespace pm {

constexpr int kIdxTile = 256;        // vertices per block = threads per block
constexpr int kIdxUnroll = 8;        // entries per thread in flight
constexpr int kIdxPairs = kCountLabels / 2;

// kSat: rows may hold more than 65,535 entries of one label; a 16-bit
// counter that already holds 255 gives its increment back, so it never
// exceeds 255 + (threads of the block) and never carries into its neighbour.
template <bool kSat>
__global__ __launch_bounds__(kIdxTile) void label_count_tiles_kernel(
    int64_t n, int64_t np, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const uint8_t *__restrict__ labels, int nlab, uint8_t *__restrict__ cnt, int64_t hub_min) {
    __shared__ uint32_t s_off[kIdxTile + 1];       // row starts relative to the tile's first entry
    __shared__ uint32_t s_h[kIdxPairs][kIdxTile];  // 16-bit counters: label L in word L / 2
    __shared__ uint64_t s_hub[kIdxTile / kWave];   // hub rows, one ballot per wavefront
    __shared__ uint32_t s_rng[2 * (kIdxTile + 1)]; // [begin, end) stretches without hub rows
    __shared__ int s_nrng;
    const int t = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * kIdxTile;
    const int64_t vend = v0 + kIdxTile < n ? v0 + kIdxTile : n;
    const int64_t e0 = rp[v0];
    s_off[t] = (uint32_t)(rp[v0 + t < vend ? v0 + t : vend] - e0);
    if (t == 0) s_off[kIdxTile] = (uint32_t)(rp[vend] - e0);
    const int npairs = (nlab + 1) >> 1;
    for (int i = 0; i < npairs; ++i) s_h[i][t] = 0;
    __syncthreads();
    const bool hub = (int64_t)(s_off[t + 1] - s_off[t]) > hub_min;
    const uint64_t hb = ballot64(hub);
    if (lane_id() == 0) s_hub[t / kWave] = hb;
    __syncthreads();
    if (t == 0) {
        // the tile's stretch with the hub rows cut out
        int nr = 0;
        uint32_t from = 0;
        for (int w = 0; w < kIdxTile / kWave; ++w)
            for (uint64_t m = s_hub[w]; m; m &= m - 1) {
                const int r = w * kWave + __builtin_ctzll(m);
                if (s_off[r] > from) {
                    s_rng[2 * nr] = from;
                    s_rng[2 * nr + 1] = s_off[r];
                    ++nr;
                }
                from = s_off[r + 1];
            }
        if (s_off[kIdxTile] > from) {
            s_rng[2 * nr] = from;
            s_rng[2 * nr + 1] = s_off[kIdxTile];
            ++nr;
        }
        s_nrng = nr;
    }
    __syncthreads();
    const int nr = s_nrng;
    const int32_t *__restrict__ tcol = col + e0;
    for (int ri = 0; ri < nr; ++ri) {
        const uint32_t lo = s_rng[2 * ri], hi = s_rng[2 * ri + 1];
        for (uint32_t base = lo; base < hi; base += kIdxTile * kIdxUnroll) {
            uint32_t k[kIdxUnroll];
            int32_t c[kIdxUnroll];
#pragma unroll
            for (int u = 0; u < kIdxUnroll; ++u) {
                k[u] = base + (uint32_t)(u * kIdxTile + t);
                c[u] = __builtin_nontemporal_load(tcol + (k[u] < hi ? k[u] : hi - 1));
            }
            int lab[kIdxUnroll];
#pragma unroll
            for (int u = 0; u < kIdxUnroll; ++u) lab[u] = labels[c[u]];
#pragma unroll
            for (int u = 0; u < kIdxUnroll; ++u) {
                if (k[u] >= hi || lab[u] >= nlab) continue;
                // last row whose start is <= k (empty rows share starts)
                int a = 0, b = kIdxTile + 1;
                while (b - a > 1) {
                    const int mid = (a + b) >> 1;
                    if (s_off[mid] <= k[u]) a = mid;
                    else b = mid;
                }
                const int sh = (lab[u] & 1) * 16;
                if (kSat) {
                    const uint32_t was = atomicAdd(&s_h[lab[u] >> 1][a], 1u << sh);
                    if (((was >> sh) & 0xffffu) >= 255u) atomicSub(&s_h[lab[u] >> 1][a], 1u << sh);
                } else {
                    atomicAdd(&s_h[lab[u] >> 1][a], 1u << sh);
                }
            }
        }
    }
    __syncthreads();
    // saturated counts, label by label: 64 threads write a label's 256
    // bytes as 4-byte words (hub rows' bytes are rewritten by the hub pass)
    for (int idx = t; idx < nlab * (kIdxTile / 4); idx += kIdxTile) {
        const int L = idx / (kIdxTile / 4), j = idx % (kIdxTile / 4);
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w = s_h[L >> 1][4 * j + i];
            const uint32_t cc = (L & 1) ? (w >> 16) : (w & 0xffffu);
            o |= (cc > 255u ? 255u : cc) << (8 * i);
        }
        *reinterpret_cast<uint32_t *>(cnt + (int64_t)L * np + v0 + 4 * j) = o;
    }
}

// One wavefront per hub segment; per-wavefront LDS counters, then one global
// atomic per (segment, label) with a non-zero count.
__global__ __launch_bounds__(kIdxTile) void label_count_hub_kernel(
    CountIndexHubs h, const int32_t *__restrict__ col, const uint8_t *__restrict__ labels,
    int nlab) {
    __shared__ uint32_t s_c[kIdxTile / kWave][kCountLabels];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int64_t seg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (seg >= h.n_segs) return;
    s_c[wib][lane] = 0;
    __builtin_amdgcn_wave_barrier();
    const int64_t b = h.seg_b[seg], e = h.seg_e[seg];
    for (int64_t k0 = b; k0 < e; k0 += (int64_t)kWave * kIdxUnroll) {
        int32_t c[kIdxUnroll];
        bool in[kIdxUnroll];
#pragma unroll
        for (int u = 0; u < kIdxUnroll; ++u) {
            const int64_t k = k0 + (int64_t)u * kWave + lane;
            in[u] = k < e;
            c[u] = __builtin_nontemporal_load(col + (in[u] ? k : e - 1));
        }
        int lab[kIdxUnroll];
#pragma unroll
        for (int u = 0; u < kIdxUnroll; ++u) lab[u] = labels[c[u]];
#pragma unroll
        for (int u = 0; u < kIdxUnroll; ++u)
            if (in[u] && lab[u] < nlab) atomicAdd(&s_c[wib][lab[u]], 1u);
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t mine = s_c[wib][lane];
    if (lane < nlab && mine)
        atomicAdd(h.hub_cnt + (int64_t)h.seg_slot[seg] * kCountLabels + lane, mine);
}

__global__ __launch_bounds__(kIdxTile) void label_count_hub_store_kernel(CountIndexHubs h,
                                                                         int64_t np, int nlab,
                                                                         uint8_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.n_hubs * kCountLabels) return;
    const int64_t slot = i / kCountLabels;
    const int L = (int)(i % kCountLabels);
    if (L >= nlab) return;
    const uint32_t c = h.hub_cnt[i];
    cnt[(int64_t)L * np + h.hub_v[slot]] = (uint8_t)(c > 255u ? 255u : c);
}

void launch_label_count(hipStream_t s, int64_t n, int64_t np, const int64_t *rp,
                        const int32_t *col, const uint8_t *labels, int nlab, uint8_t *cnt,
                        const CountIndexHubs &h) {
    if (n <= 0) return;
    const int64_t tiles = (n + kIdxTile - 1) / kIdxTile;
    hipLaunchKernelGGL(label_count_tiles_kernel<false>, dim3((unsigned)tiles), dim3(kIdxTile), 0, s,
                       n, np, rp, col, labels, nlab, cnt, (int64_t)kBinWaveMaxDeg);
    if (h.n_segs > 0) {
        launch_fill_i32(s, reinterpret_cast<int32_t *>(h.hub_cnt), h.n_hubs * kCountLabels, 0);
        hipLaunchKernelGGL(label_count_hub_kernel,
                           dim3((unsigned)((h.n_segs * kWave + kIdxTile - 1) / kIdxTile)),
                           dim3(kIdxTile), 0, s, h, col, labels, nlab);
        hipLaunchKernelGGL(label_count_hub_store_kernel,
                           dim3((unsigned)((h.n_hubs * kCountLabels + kIdxTile - 1) / kIdxTile)),
                           dim3(kIdxTile), 0, s, h, np, nlab, cnt);
    }
}

// Every row in the tiles, with saturating counters (no hub pass): for a
// subgraph whose rows are short enough that a tile's stretch stays below
// 2^32 entries, such as the label-pair subgraph.
void launch_label_count_rows(hipStream_t s, int64_t n, int64_t np, const int64_t *rp,
                             const int32_t *col, const uint8_t *labels, int nlab, uint8_t *cnt) {
    if (n <= 0) return;
    const int64_t tiles = (n + kIdxTile - 1) / kIdxTile;
    hipLaunchKernelGGL(label_count_tiles_kernel<true>, dim3((unsigned)tiles), dim3(kIdxTile), 0, s,
                       n, np, rp, col, labels, nlab, cnt, INT64_MAX);
}

}  // namespace pm
