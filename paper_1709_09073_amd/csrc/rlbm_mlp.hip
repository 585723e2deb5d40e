// rlbm_mlp.hip -- forward, backward and Adam kernels of the inversion-guess
// network (see rlbm_mlp.h for the architecture and weight layout).  Gradients are
// formed per sample and summed column by column in a fixed order, so a call gives
// the same bits every time.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "rlbm.h"
#include "rlbm_mlp.h"

namespace {

using namespace rlbm_mlp;

constexpr int BLOCK = 256;

// Workspace layout (floats): per-sample gradient columns G[(NTRAIN + 1) x n] (the
// last column holds the per-sample loss), the summed gradient and loss
// (NTRAIN + 1), Adam's first and second moments (NTRAIN each), init statistics (4),
// then, 8-byte aligned, the first-stage column sums in double ((NTRAIN + 1) x PARTS).
struct Workspace {
    float *G, *grad, *m, *v, *stats;
    double *partial;   // (NTRAIN + 1) x PARTS first-stage sums
};

Workspace carve(void *ws, long long n) {
    float *p = static_cast<float *>(ws);
    Workspace w;
    w.G = p;
    w.grad = w.G + (long long)(NTRAIN + 1) * n;
    w.m = w.grad + (NTRAIN + 1);
    w.v = w.m + NTRAIN;
    w.stats = w.v + NTRAIN;
    // 8-byte aligned start for the partial sums
    uintptr_t q = reinterpret_cast<uintptr_t>(w.stats + 4);
    q = (q + 7) & ~uintptr_t(7);
    w.partial = reinterpret_cast<double *>(q);
    return w;
}

// d(loss)/d(params) of one sample, loss = mean_i (y_i - tn_i)^2, tn = (t - m)/s.
__global__ __launch_bounds__(BLOCK) void k_sample_grads(const float *__restrict__ w, const float *__restrict__ x,
                                                        const float *__restrict__ t, long long n,
                                                        float *__restrict__ G) {
    const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const float xh = (x[i] - w[0]) * w[1];
    const float tn = (t[i] - w[2]) / w[3];
    float z[H];
    float y = w[HDR + 3 * H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        z[h] = w[HDR + h] * xh + w[HDR + H + h];
        y += w[HDR + 2 * H + h] * fmaxf(z[h], 0.0f);
    }
    const float r = y - tn;
    const float inv_n = 1.0f / (float)n;
    const float dy = 2.0f * r * inv_n;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const float act = fmaxf(z[h], 0.0f);
        const float dz = z[h] > 0.0f ? dy * w[HDR + 2 * H + h] : 0.0f;
        G[(long long)h * n + i] = dz * xh;                 // W1_h
        G[(long long)(H + h) * n + i] = dz;                // b1_h
        G[(long long)(2 * H + h) * n + i] = dy * act;      // W2_h
    }
    G[(long long)(3 * H) * n + i] = dy;                    // b2
    G[(long long)NTRAIN * n + i] = r * r * inv_n;          // loss share
}

constexpr int PARTS = 64;   // workgroups per column in the first reduction stage

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sm[BLOCK];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int st = BLOCK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
        __syncthreads();
    }
    return sm[0];
}

// Stage 1: partial[c][p] = sum of G[c][i] over the p-th contiguous chunk of i
// (grid: PARTS x columns).  Stage 2: out[c] = sum_p partial[c][p].  Both stages sum
// in a fixed order, so the result does not depend on scheduling.
__global__ __launch_bounds__(BLOCK) void k_column_partials(const float *__restrict__ G, long long n,
                                                           double *__restrict__ partial) {
    const int part = blockIdx.x, c = blockIdx.y;
    const long long chunk = (n + PARTS - 1) / PARTS;
    const long long lo = part * chunk, hi = lo + chunk < n ? lo + chunk : n;
    const float *col = G + (long long)c * n;
    double acc = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += BLOCK) acc += (double)col[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partial[(long long)c * PARTS + part] = s;
}

__global__ __launch_bounds__(BLOCK) void k_column_final(const double *__restrict__ partial, float *__restrict__ out) {
    const double s = block_sum(threadIdx.x < PARTS ? partial[(long long)blockIdx.x * PARTS + threadIdx.x] : 0.0);
    if (threadIdx.x == 0) out[blockIdx.x] = (float)s;
}

__global__ void k_fill(float *p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One Adam step on the trainable part of w (bias-corrected moments).
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int step, float lr, float *loss_out) {
    const int j = threadIdx.x;
    if (j == 0 && loss_out) loss_out[step - 1] = grad[NTRAIN];
    if (j >= NTRAIN) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[j];
    const float mj = b1 * m[j] + (1.0f - b1) * g;
    const float vj = b2 * v[j] + (1.0f - b2) * g * g;
    m[j] = mj;
    v[j] = vj;
    const float mh = mj / (1.0f - powf(b1, (float)step));
    const float vh = vj / (1.0f - powf(b2, (float)step));
    w[HDR + j] -= lr * mh / (sqrtf(vh) + eps);
}

// min/max of x and mean/std of t (one workgroup, fixed order), then the initial weights.
__global__ __launch_bounds__(BLOCK) void k_init(float *__restrict__ w, const float *__restrict__ x,
                                                const float *__restrict__ t, long long n,
                                                const float *__restrict__ noise) {
    double lo = 1e300, hi = -1e300, s1 = 0.0, s2 = 0.0;
    for (long long i = threadIdx.x; i < n; i += BLOCK) {
        const double xv = x[i], tv = t[i];
        lo = fmin(lo, xv);
        hi = fmax(hi, xv);
        s1 += tv;
        s2 += tv * tv;
    }
    __shared__ double sl[BLOCK], sh[BLOCK], a1[BLOCK], a2[BLOCK];
    sl[threadIdx.x] = lo;
    sh[threadIdx.x] = hi;
    a1[threadIdx.x] = s1;
    a2[threadIdx.x] = s2;
    __syncthreads();
    for (int st = BLOCK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + st]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
            a1[threadIdx.x] += a1[threadIdx.x + st];
            a2[threadIdx.x] += a2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double span = sh[0] - sl[0];
        const double mean = a1[0] / (double)n;
        const double var = fmax(a2[0] / (double)n - mean * mean, 0.0);
        w[0] = (float)(0.5 * (sh[0] + sl[0]));
        w[1] = (float)(span > 0.0 ? 2.0 / span : 1.0);
        w[2] = (float)mean;
        w[3] = (float)(var > 0.0 ? sqrt(var) : 1.0);
        for (int h = 0; h < H; ++h) {
            w[HDR + h] = 1.0f;
            w[HDR + H + h] = -(-1.0f + 2.0f * (h + 0.5f) / H);
            w[HDR + 2 * H + h] = 0.1f * noise[h];
        }
        w[HDR + 3 * H] = 0.1f * noise[H];
    }
}

__global__ __launch_bounds__(BLOCK) void k_predict(const float *__restrict__ w, const float *__restrict__ x,
                                                   float *__restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) y[i] = eval(w, x[i]);
}

unsigned blocks_for(long long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

int loss_grad_enqueue(const float *w, const float *x, const float *t, long long n, const Workspace &ws,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_sample_grads, dim3(blocks_for(n)), dim3(BLOCK), 0, s, w, x, t, n, ws.G);
    hipLaunchKernelGGL(k_column_partials, dim3(PARTS, NTRAIN + 1), dim3(BLOCK), 0, s, ws.G, n, ws.partial);
    hipLaunchKernelGGL(k_column_final, dim3(NTRAIN + 1), dim3(BLOCK), 0, s, ws.partial, ws.grad);
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

constexpr uint64_t workspace_bytes(int64_t n) {
    return sizeof(float) * ((uint64_t)(NTRAIN + 1) * (uint64_t)(n + 1) + 2u * NTRAIN + 4u) + 8u +
           sizeof(double) * (uint64_t)(NTRAIN + 1) * PARTS;
}

// Workspace of the allocation-free training call: a device array of fixed size, one
// per GPU for the life of the process, laid out by carve() like a caller's workspace
// (training on n <= RLBM_MLP_NOALLOC_MAX samples uses a prefix of it).
constexpr uint64_t SCRATCH_BYTES = workspace_bytes(RLBM_MLP_NOALLOC_MAX);
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Device address of `scratch` on the current device, looked up once per device (the
// host-side name is only a stand-in for the symbol, never a device address).
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_addr[MAX_DEVICES] = {};

void *scratch_on_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        scratch_addr[dev] = ptr;
    }
    return scratch_addr[dev];
}

}  // namespace

extern "C" {

uint64_t rlbm_mlp_workspace_bytes(int64_t n) {
    if (n < 1) return 0;
    return workspace_bytes(n);
}

int rlbm_mlp_init(float *w, const float *x, const float *t, int64_t n, const float *noise, void *workspace,
                  void *stream) {
    if (!w || !x || !t || !noise || n < 2) return RLBM_EINVAL;
    (void)workspace;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(BLOCK), 0, (hipStream_t)stream, w, x, t, (long long)n, noise);
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

int rlbm_mlp_loss_grad(const float *w, const float *x, const float *t, int64_t n, float *grad, float *loss,
                       void *workspace, void *stream) {
    if (!w || !x || !t || !grad || !loss || !workspace || n < 1) return RLBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Workspace ws = carve(workspace, n);
    int rc = loss_grad_enqueue(w, x, t, n, ws, s);
    if (rc) return rc;
    if (hipMemcpyAsync(grad, ws.grad, sizeof(float) * NTRAIN, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(loss, ws.grad + NTRAIN, sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return RLBM_EHIP;
    return RLBM_OK;
}

int rlbm_mlp_train(float *w, const float *x, const float *t, int64_t n, int32_t iters, float lr, float *loss_out,
                   void *workspace, void *stream) {
    if (!w || !x || !t || !workspace || n < 1 || iters < 0 || !(lr > 0.0f)) return RLBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Workspace ws = carve(workspace, n);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(2 * NTRAIN), 0, s, ws.m, 2 * NTRAIN, 0.0f);
    for (int it = 1; it <= iters; ++it) {
        int rc = loss_grad_enqueue(w, x, t, n, ws, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_adam, dim3(1), dim3(128), 0, s, w, ws.grad, ws.m, ws.v, it, lr, loss_out);
    }
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

int rlbm_mlp_train_noalloc(float *w, const float *x, const float *t, int64_t n, int32_t iters, float lr,
                           float *loss_out, void *stream) {
    if (!w || !x || !t || n < 1 || n > RLBM_MLP_NOALLOC_MAX || iters < 0 || !(lr > 0.0f)) return RLBM_EINVAL;
    void *ws = scratch_on_current_device();
    if (!ws) return RLBM_EHIP;
    return rlbm_mlp_train(w, x, t, n, iters, lr, loss_out, ws, stream);
}

int rlbm_mlp_predict(const float *w, const float *x, float *y, int64_t n, void *stream) {
    if (!w || !x || !y || n < 0) return RLBM_EINVAL;
    if (n == 0) return RLBM_OK;
    hipLaunchKernelGGL(k_predict, dim3(blocks_for(n)), dim3(BLOCK), 0, (hipStream_t)stream, w, x, y, (long long)n);
    return hipGetLastError() == hipSuccess ? RLBM_OK : RLBM_EHIP;
}

}  // extern "C"
