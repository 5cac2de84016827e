// Learned ordering of the non-local constraints: active role totals, the
// per-constraint features, the perceptron's forward pass, its loss gradient
// and the Adam update, all in fp32.  The paper orders constraints by fixed
// heuristics (ordering heuristics of the constraint generation section) and
// leaves selection and ordering by a model open (conclusion); the features
// and the model are defined with PM_ORDER_LEARNED in pm.h.
//
// The model is tiny (5122 parameters, at most 64 constraints per choice), so
// every kernel works on tiles of 64 samples in LDS: W2 is staged with rows
// padded to 65 floats so that lanes reading one column hit distinct banks,
// activations are stored the same way, and each thread of the gradient
// kernel owns a fixed set of parameters whose sums it keeps in registers
// across tiles; partial sums per block are added in a fixed order, so the
// gradient does not depend on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_util.h"
#include "pm_internal.h"

namespace pm {
namespace {

constexpr int kOB = 256;              // threads per block of the model kernels
constexpr int kTile = 64;             // samples per tile (>= PM_MAX_CONSTRAINTS)
constexpr int kPad = kMlpHid + 1;     // padded row stride of 64-wide LDS matrices
constexpr int kPer = (kMlpParams + kOB - 1) / kOB;   // parameters per thread

template <typename M>
__global__ __launch_bounds__(256) void role_totals_kernel(const int32_t *__restrict__ tasks,
                                                          int64_t n_tasks,
                                                          const M *__restrict__ omega, int n0,
                                                          unsigned long long *counts) {
    __shared__ unsigned int sc[kMaxK];
    for (int i = threadIdx.x; i < kMaxK; i += blockDim.x) sc[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop bound is uniform over the block, so every lane takes part in
    // the ballots
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n_tasks; base += stride) {
        const int64_t i = base + threadIdx.x;
        const uint64_t r = i < n_tasks ? (uint64_t)omega[tasks[i]] : 0ull;
        for (int q = 0; q < n0; ++q) {
            const uint64_t b = ballot64(((r >> q) & 1ull) != 0);
            if (lane_id() == 0 && b) atomicAdd(&sc[q], (unsigned int)__popcll(b));
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n0; q += blockDim.x)
        if (sc[q]) atomicAdd(counts + q, (unsigned long long)sc[q]);
}

__device__ void load_w2(const float *__restrict__ w, float *sW2) {
    for (int i = threadIdx.x; i < kMlpHid * kMlpHid; i += blockDim.x)
        sW2[(i / kMlpHid) * kPad + (i % kMlpHid)] = w[kOffW2 + i];
}

// Forward pass of `rows` (<= kTile) samples held in sX[kTile][kMlpIn]; sH1
// and sH2 ([kTile][kPad]) receive the ReLU activations (0 for rows >=
// rows), sY ([kTile][kMlpOut]) the outputs.  Every thread of the block takes
// part; ends with a barrier.
__device__ void tile_forward(const float *__restrict__ w, const float *sW2, const float *sX,
                             float *sH1, float *sH2, float *sY, int rows) {
    const int tid = threadIdx.x;
    for (int o = tid; o < kTile * kMlpHid; o += blockDim.x) {
        const int r = o / kMlpHid, j = o % kMlpHid;
        float z = w[kOffB1 + j];
#pragma unroll
        for (int f = 0; f < kMlpIn; ++f) z = fmaf(w[kOffW1 + j * kMlpIn + f], sX[r * kMlpIn + f], z);
        sH1[r * kPad + j] = r < rows ? fmaxf(z, 0.0f) : 0.0f;
    }
    __syncthreads();
    for (int o = tid; o < kTile * kMlpHid; o += blockDim.x) {
        const int r = o / kMlpHid, j = o % kMlpHid;
        float z = w[kOffB2 + j];
#pragma unroll 16
        for (int k = 0; k < kMlpHid; ++k) z = fmaf(sW2[j * kPad + k], sH1[r * kPad + k], z);
        sH2[r * kPad + j] = r < rows ? fmaxf(z, 0.0f) : 0.0f;
    }
    __syncthreads();
    for (int o = tid; o < kTile * kMlpOut; o += blockDim.x) {
        const int r = o / kMlpOut, j = o % kMlpOut;
        float z = w[kOffB3 + j];
#pragma unroll 16
        for (int k = 0; k < kMlpHid; ++k) z = fmaf(w[kOffW3 + j * kMlpHid + k], sH2[r * kPad + k], z);
        sY[r * kMlpOut + j] = z;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kOB) void mlp_forward_kernel(const float *__restrict__ w,
                                                          const float *__restrict__ x, int64_t n,
                                                          float *__restrict__ y) {
    __shared__ float sW2[kMlpHid * kPad];
    __shared__ float sX[kTile * kMlpIn];
    __shared__ float sH1[kTile * kPad];
    __shared__ float sH2[kTile * kPad];
    __shared__ float sY[kTile * kMlpOut];
    load_w2(w, sW2);
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < n; t0 += (int64_t)gridDim.x * kTile) {
        const int rows = (int)(n - t0 < kTile ? n - t0 : kTile);
        __syncthreads();
        for (int i = threadIdx.x; i < kTile * kMlpIn; i += blockDim.x)
            sX[i] = i < rows * kMlpIn ? x[t0 * kMlpIn + i] : 0.0f;
        __syncthreads();
        tile_forward(w, sW2, sX, sH1, sH2, sY, rows);
        for (int i = threadIdx.x; i < rows * kMlpOut; i += blockDim.x) y[t0 * kMlpOut + i] = sY[i];
    }
}

// Partial gradients of L = sum (y - t)^2 / (2n) over the tiles this block
// takes (tiles blockIdx.x, blockIdx.x + gridDim.x, ...), by the chain rule:
// dL/dy = (y - t)/n, delta2 = (W3^T dL/dy) * [h2 > 0], delta1 = (W2^T delta2)
// * [h1 > 0]; weight gradients are sums over samples of delta (outer) input.
__global__ __launch_bounds__(kOB) void mlp_grad_kernel(const float *__restrict__ w,
                                                       const float *__restrict__ x,
                                                       const float *__restrict__ t, int64_t n,
                                                       float *__restrict__ partial,
                                                       float *__restrict__ ploss) {
    __shared__ float sW2[kMlpHid * kPad];
    __shared__ float sX[kTile * kMlpIn];
    __shared__ float sH1[kTile * kPad];   // h1, then delta1
    __shared__ float sH2[kTile * kPad];   // h2, then delta2
    __shared__ float sY[kTile * kMlpOut];
    __shared__ float sD[kTile * kMlpOut]; // dL/dy
    __shared__ float sRed[kOB];
    const int tid = threadIdx.x;
    float acc[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) acc[j] = 0.0f;
    float lsum = 0.0f;
    const float inv_n = 1.0f / (float)n;
    load_w2(w, sW2);
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < n; t0 += (int64_t)gridDim.x * kTile) {
        const int rows = (int)(n - t0 < kTile ? n - t0 : kTile);
        __syncthreads();
        for (int i = tid; i < kTile * kMlpIn; i += blockDim.x)
            sX[i] = i < rows * kMlpIn ? x[t0 * kMlpIn + i] : 0.0f;
        __syncthreads();
        tile_forward(w, sW2, sX, sH1, sH2, sY, rows);
        for (int i = tid; i < kTile * kMlpOut; i += blockDim.x) {
            float d = 0.0f;
            if (i < rows * kMlpOut) {
                d = sY[i] - t[t0 * kMlpOut + i];
                lsum = fmaf(d, d, lsum);
            }
            sD[i] = d * inv_n;
        }
        __syncthreads();
        // W3, b3: sums over the tile of dL/dy (outer) h2
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int p = tid + j * kOB;
            if (p >= kOffW3 && p < kOffB3) {
                const int o = (p - kOffW3) / kMlpHid, k = (p - kOffW3) % kMlpHid;
                float s = 0.0f;
                for (int r = 0; r < kTile; ++r) s = fmaf(sD[r * kMlpOut + o], sH2[r * kPad + k], s);
                acc[j] += s;
            } else if (p >= kOffB3 && p < kMlpParams) {
                const int o = p - kOffB3;
                float s = 0.0f;
                for (int r = 0; r < kTile; ++r) s += sD[r * kMlpOut + o];
                acc[j] += s;
            }
        }
        __syncthreads();
        // delta2 in place of h2
        for (int o = tid; o < kTile * kMlpHid; o += blockDim.x) {
            const int r = o / kMlpHid, i = o % kMlpHid;
            float g = 0.0f;
            if (sH2[r * kPad + i] > 0.0f) {
#pragma unroll
                for (int oo = 0; oo < kMlpOut; ++oo)
                    g = fmaf(w[kOffW3 + oo * kMlpHid + i], sD[r * kMlpOut + oo], g);
            }
            sH2[r * kPad + i] = g;
        }
        __syncthreads();
        // W2, b2: sums of delta2 (outer) h1
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int p = tid + j * kOB;
            if (p >= kOffW2 && p < kOffB2) {
                const int jj = (p - kOffW2) / kMlpHid, k = (p - kOffW2) % kMlpHid;
                float s = 0.0f;
                for (int r = 0; r < kTile; ++r) s = fmaf(sH2[r * kPad + jj], sH1[r * kPad + k], s);
                acc[j] += s;
            } else if (p >= kOffB2 && p < kOffW3) {
                const int jj = p - kOffB2;
                float s = 0.0f;
                for (int r = 0; r < kTile; ++r) s += sH2[r * kPad + jj];
                acc[j] += s;
            }
        }
        __syncthreads();
        // delta1 in place of h1 (each element reads only its own h1)
        for (int o = tid; o < kTile * kMlpHid; o += blockDim.x) {
            const int r = o / kMlpHid, k = o % kMlpHid;
            float g = 0.0f;
            if (sH1[r * kPad + k] > 0.0f) {
#pragma unroll 16
                for (int i = 0; i < kMlpHid; ++i) g = fmaf(sW2[i * kPad + k], sH2[r * kPad + i], g);
            }
            sH1[r * kPad + k] = g;
        }
        __syncthreads();
        // W1, b1: sums of delta1 (outer) x
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int p = tid + j * kOB;
            if (p < kOffB1) {
                const int jj = p / kMlpIn, f = p % kMlpIn;
                float s = 0.0f;
                for (int r = 0; r < kTile; ++r) s = fmaf(sH1[r * kPad + jj], sX[r * kMlpIn + f], s);
                acc[j] += s;
            } else if (p < kOffW2) {
                const int jj = p - kOffB1;
                float s = 0.0f;
                for (int r = 0; r < kTile; ++r) s += sH1[r * kPad + jj];
                acc[j] += s;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int p = tid + j * kOB;
        if (p < kMlpParams) partial[(int64_t)blockIdx.x * kMlpParams + p] = acc[j];
    }
    sRed[tid] = lsum;
    __syncthreads();
    for (int h = kOB / 2; h > 0; h >>= 1) {
        if (tid < h) sRed[tid] += sRed[tid + h];
        __syncthreads();
    }
    if (tid == 0) ploss[blockIdx.x] = sRed[0];
}

// Fixed-order sums of the per-block partials.
__global__ void mlp_grad_reduce_kernel(const float *__restrict__ partial,
                                       const float *__restrict__ ploss, int nblocks, int64_t n,
                                       float *__restrict__ grad, float *__restrict__ loss) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p < kMlpParams) {
        float s = 0.0f;
        for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * kMlpParams + p];
        grad[p] = s;
    }
    if (p == 0 && loss) {
        float s = 0.0f;
        for (int b = 0; b < nblocks; ++b) s += ploss[b];
        loss[0] = s / (2.0f * (float)n);
    }
}

// Adam (Kingma and Ba, Algorithm 1): bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ grad,
                            float *__restrict__ m, float *__restrict__ v, float lr, float bc1,
                            float bc2) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mm = 0.9f * m[p] + 0.1f * g;
    const float vv = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mm;
    v[p] = vv;
    w[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

// Features of every constraint at the current state, model outputs, and the
// greedy choice among the remaining ones (or the forced constraint).
__global__ __launch_bounds__(kOB) void order_select_kernel(OrderArgs a, OrderPick *out) {
    __shared__ float sW2[kMlpHid * kPad];
    __shared__ float sX[kTile * kMlpIn];
    __shared__ float sH1[kTile * kPad];
    __shared__ float sH2[kTile * kPad];
    __shared__ float sY[kTile * kMlpOut];
    __shared__ float lgc[kMaxK], lgc0[kMaxK], lgF[kMaxK];
    const int tid = threadIdx.x;
    if (tid < kMaxK) {
        const bool in = tid < a.n0;
        lgc[tid] = in ? log2f(1.0f + (float)a.counts[tid]) : 0.0f;
        lgc0[tid] = in ? log2f(1.0f + (float)a.counts0[tid]) : 0.0f;
        lgF[tid] = in ? log2f(1.0f + (float)a.role_freq[tid]) : 0.0f;
    }
    if (a.w) load_w2(a.w, sW2);
    __syncthreads();
    const float lg_active = log2f(1.0f + (float)a.n_active);
    for (int r = tid; r < kTile; r += blockDim.x) {
        float f[kMlpIn];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) f[i] = 0.0f;
        if (r < a.n_cons) {
            const ConstraintDesc d = a.cons[r];
            const int nv = __popcll(d.vmask);
            float mn = INFINITY, mx = -INFINITY, sum = 0.0f, sumF = 0.0f, sumD = 0.0f;
            for (uint64_t b = d.vmask; b; b &= b - 1) {
                const int q = __ffsll((unsigned long long)b) - 1;
                const float l = lgc[q];
                mn = fminf(mn, l);
                mx = fmaxf(mx, l);
                sum += l;
                sumF += lgF[q];
                sumD += lgc0[q] - l;
            }
            const float inv = nv ? 1.0f / (float)nv : 0.0f;
            f[0] = (float)d.n_edges / 8.0f;
            f[1] = (float)nv / 8.0f;
            f[2] = (d.kind == 0 || d.kind == 2) ? 1.0f : 0.0f;
            f[3] = (d.kind == 2 || d.kind == 3) ? 1.0f : 0.0f;
            f[4] = (float)__popcll(d.heads & d.vmask) * inv;
            f[5] = nv ? mn / 16.0f : 0.0f;
            f[6] = sum * inv / 16.0f;
            f[7] = nv ? mx / 16.0f : 0.0f;
            f[8] = lg_active / 16.0f;
            f[9] = sumF * inv / 16.0f;
            f[10] = sumD * inv / 16.0f;
            f[11] = (float)a.done / (float)a.n_cons;
        }
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) sX[r * kMlpIn + i] = f[i];
    }
    __syncthreads();
    if (a.w) tile_forward(a.w, sW2, sX, sH1, sH2, sY, a.n_cons);
    if (tid == 0) {
        int idx = -1;
        float best = -INFINITY;
        if (a.forced >= 0 && a.forced < a.n_cons) {
            idx = a.forced;
            best = a.w ? sY[idx * kMlpOut] - sY[idx * kMlpOut + 1] : 0.0f;
        } else if (a.forced < 0) {
            for (int r = 0; r < a.n_cons; ++r) {
                if (!((a.remaining >> r) & 1ull)) continue;
                float s = a.w ? sY[r * kMlpOut] - sY[r * kMlpOut + 1] : 0.0f;
                if (!(s == s)) s = -INFINITY;    // NaN ranks last
                if (idx < 0 || s > best) {
                    idx = r;
                    best = s;
                }
            }
        }
        OrderPick p;
        p.idx = idx;
        p.score = best;
        for (int i = 0; i < kMlpOut; ++i) p.pred[i] = (a.w && idx >= 0) ? sY[idx * kMlpOut + i] : 0.0f;
        for (int i = 0; i < kMlpIn; ++i) p.feat[i] = idx >= 0 ? sX[idx * kMlpIn + i] : 0.0f;
        unsigned long long roles = 0;
        for (int q = 0; q < a.n0; ++q) roles += a.counts[q];
        p.roles = roles;
        *out = p;
    }
}

}  // namespace

template <typename M>
void launch_role_totals(hipStream_t s, const int32_t *tasks, int64_t n_tasks, const M *omega,
                        int n0, unsigned long long *counts) {
    if (n_tasks <= 0) return;
    int64_t g = (n_tasks + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(role_totals_kernel<M>, dim3((unsigned)g), dim3(256), 0, s, tasks, n_tasks,
                       omega, n0, counts);
}

#define PM_INST(M)                                                                           \
    template void launch_role_totals<M>(hipStream_t, const int32_t *, int64_t, const M *, int, \
                                        unsigned long long *);
PM_INST(uint8_t)
PM_INST(uint16_t)
PM_INST(uint32_t)
PM_INST(uint64_t)
#undef PM_INST

void launch_order_select(hipStream_t s, const OrderArgs &a, OrderPick *out) {
    hipLaunchKernelGGL(order_select_kernel, dim3(1), dim3(kOB), 0, s, a, out);
}

void launch_mlp_forward(hipStream_t s, const float *w, const float *x, int64_t n, float *y) {
    if (n <= 0) return;
    int64_t g = (n + kTile - 1) / kTile;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)g), dim3(kOB), 0, s, w, x, n, y);
}

void launch_mlp_grad(hipStream_t s, const float *w, const float *x, const float *t, int64_t n,
                     float *partial, float *partial_loss, float *grad, float *loss) {
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(kMlpGradGrid), dim3(kOB), 0, s, w, x, t, n, partial,
                       partial_loss);
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s,
                       partial, partial_loss, kMlpGradGrid, n, grad, loss);
}

void launch_adam(hipStream_t s, float *w, const float *grad, float *m, float *v, float lr,
                 float bc1, float bc2) {
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, w, grad, m,
                       v, lr, bc1, bc2);
}

}  // namespace pm
