// State import and reuse kernels for gfx950, and the static scratch array of
// the no-allocation prune.
//
// The pruning state is the role-set array omega; the edge state is derived
// from it.  Any state that still holds the complete set is a valid place to
// (re)start the constraint-checking loop -- the checkpoint-and-resume of the
// paper's load-balancing subsection, and the candidate set and solution
// reuse of its interactive incremental search.  These kernels bring such a
// state in (omega &= state), seed the final search with roles and edges
// already known to be in the complete set, and give the per-label degree
// sums that bound scratch sizes.
#include <mutex>

#include "device_util.h"
#include "pm_internal.h"

namespace pm {

constexpr int kStateBlock = 256;

static int64_t grid_for(int64_t n, int64_t cap = 8192) {
    int64_t g = (n + kStateBlock - 1) / kStateBlock;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

// omega(v) &= state(v) over all vertices.
template <typename M>
__global__ __launch_bounds__(kStateBlock) void and_state_kernel(int64_t n, M *omega,
                                                                const uint64_t *state) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const M w = omega[v];
        if (w) omega[v] = (M)((uint64_t)w & state[v]);
    }
}

template <typename M>
void launch_and_state(hipStream_t s, int64_t n, M *omega, const uint64_t *state) {
    if (n <= 0) return;
    hipLaunchKernelGGL(and_state_kernel<M>, dim3((unsigned)grid_for(n)), dim3(kStateBlock), 0, s,
                       n, omega, state);
}

// cert(v) = known(v) & omega(v) for the vertices of the task list (the
// others are not read by the final search).
template <typename M>
__global__ __launch_bounds__(kStateBlock) void known_roles_kernel(const int32_t *tasks,
                                                                  int64_t n_tasks, const M *omega,
                                                                  const uint64_t *known, M *cert) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tasks;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = tasks[t];
        cert[v] = (M)((uint64_t)omega[v] & known[v]);
    }
}

template <typename M>
void launch_known_roles(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const M *omega,
                        const uint64_t *known, M *cert) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(known_roles_kernel<M>, dim3((unsigned)grid_for(n_tasks)), dim3(kStateBlock),
                       0, s, tasks, n_tasks, omega, known, cert);
}

// Certified-entry bits of the compacted subgraph from known edge bits of
// the original CSR: compacted entry k (row c_own[k], offset c_off[k] in the
// original row) is certified iff its original entry's bit is set.  One
// thread per compacted entry; a wavefront's 64 entries are one aligned word
// of c_cert, set with one atomic OR of the wavefront's ballot.
__global__ __launch_bounds__(kStateBlock) void known_edges_kernel(
    int64_t c_m, const int32_t *__restrict__ c_own, const int32_t *__restrict__ c_off,
    const int64_t *__restrict__ rp, const uint64_t *__restrict__ known, uint64_t *c_cert) {
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < c_m;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = base + threadIdx.x;
        bool on = false;
        if (k < c_m) {
            const int64_t e = rp[c_own[k]] + c_off[k];
            on = (known[e >> 6] >> (e & 63)) & 1ull;
        }
        const uint64_t b = ballot64(on);
        // wavefronts start at multiples of 64 entries: one word each
        if (lane_id() == 0 && b) atomicOr((unsigned long long *)(c_cert + (k >> 6)), b);
    }
}

void launch_known_edges(hipStream_t s, int64_t c_m, const int32_t *c_own, const int32_t *c_off,
                        const int64_t *rp, const uint64_t *known, uint64_t *c_cert) {
    if (c_m <= 0) return;
    hipLaunchKernelGGL(known_edges_kernel, dim3((unsigned)grid_for(c_m, 16384)),
                       dim3(kStateBlock), 0, s, c_m, c_own, c_off, rp, known, c_cert);
}

// Unions over the templates of one call: dst |= src, word by word.  Atomic,
// since templates pruned on concurrent streams share dst; a word whose src
// is zero is not touched.
__global__ __launch_bounds__(kStateBlock) void or_into_kernel(int64_t n, const uint64_t *src,
                                                              uint64_t *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = src[i];
        if (x) atomicOr((unsigned long long *)(dst + i), (unsigned long long)x);
    }
}

void launch_or_into(hipStream_t s, int64_t n, const uint64_t *src, uint64_t *dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(or_into_kernel, dim3((unsigned)grid_for(n)), dim3(kStateBlock), 0, s, n,
                       src, dst);
}

// Sum of degrees per label (labels below hist_len): bounds the entries of
// the candidate subgraph of a template from its labels alone.  8-bit labels
// accumulate in LDS, one global atomic per label and block.
__global__ __launch_bounds__(kStateBlock) void label_degsum_kernel(int64_t n, const int64_t *rp,
                                                                   const void *labels,
                                                                   int label_bytes,
                                                                   unsigned long long *sum,
                                                                   int64_t hist_len) {
    __shared__ unsigned long long local[256];
    const bool small = label_bytes == 1 && hist_len <= 256;
    if (small) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) local[i] = 0;
        __syncthreads();
    }
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t L = label_bytes == 1 ? (int64_t)((const uint8_t *)labels)[v]
                                           : (int64_t)((const uint16_t *)labels)[v];
        const int64_t d = rp[v + 1] - rp[v];
        if (L < hist_len && d) {
            if (small) atomicAdd(&local[L], (unsigned long long)d);
            else atomicAdd(&sum[L], (unsigned long long)d);
        }
    }
    if (small) {
        __syncthreads();
        for (int i = threadIdx.x; i < 256; i += blockDim.x)
            if (local[i]) atomicAdd(&sum[i], local[i]);
    }
}

void launch_label_degsum(hipStream_t s, int64_t n, const int64_t *rp, const void *labels,
                         int label_bytes, unsigned long long *sum, int64_t hist_len) {
    if (n <= 0) return;
    hipLaunchKernelGGL(label_degsum_kernel, dim3((unsigned)grid_for(n, 4096)), dim3(kStateBlock),
                       0, s, n, rp, labels, label_bytes, sum, hist_len);
}

// ---- static scratch of the no-allocation prune -------------------------------
// One array per device, held until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

#define PM_INSTANTIATE_STATE(M)                                                                 \
    template void launch_and_state<M>(hipStream_t, int64_t, M *, const uint64_t *);             \
    template void launch_known_roles<M>(hipStream_t, const int32_t *, int64_t, const M *,       \
                                        const uint64_t *, M *);

PM_INSTANTIATE_STATE(uint8_t)
PM_INSTANTIATE_STATE(uint16_t)
PM_INSTANTIATE_STATE(uint32_t)
PM_INSTANTIATE_STATE(uint64_t)

}  // namespace pm
