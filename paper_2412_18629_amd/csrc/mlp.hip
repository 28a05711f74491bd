// mlp.hip -- the linking-length proposer: a 24 -> 64 -> 64 -> 1 ReLU network
// that predicts ln(l) of a node from 24 summary features.  Training kernels
// (fp32 forward, backward, Adam) and the node inference kernel (bf16 weights
// and activations, fp32 accumulation) are all here; nothing in this file
// decides a result of the method: a proposal only chooses the bracket that
// the exact counting step then verifies.
//
// Parameter layout (fp32, 5825 values): W1[64][24], b1[64], W2[64][64],
// b2[64], W3[64], b3[1].  Features are standardised with a per-feature mean
// and standard deviation kept beside the parameters.
#include "common.h"
#include "phase_common.h"

namespace rs {

constexpr int NIN = RS_NFEAT, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH,
              NPARAM = OFF_B3 + 1;
static_assert(NPARAM == 5825, "parameter count");

// forward of one sample, keeping the hidden activations
__global__ void __launch_bounds__(256)
k_mlp_fwd(const float* __restrict__ p, const float* __restrict__ X, int64_t n,
          float* __restrict__ H1, float* __restrict__ H2, float* __restrict__ Y) {
    __shared__ float w[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += 256) w[i] = p[i];
    __syncthreads();
    int64_t s = blockIdx.x * 256ll + threadIdx.x;
    if (s >= n) return;
    float x[NIN], h1[NH];
#pragma unroll
    for (int i = 0; i < NIN; i++) x[i] = X[s * NIN + i];
    for (int j = 0; j < NH; j++) {
        float a = w[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < NIN; i++) a += w[OFF_W1 + j * NIN + i] * x[i];
        h1[j] = a > 0.0f ? a : 0.0f;
        H1[s * NH + j] = h1[j];
    }
    float y = w[OFF_B3];
    for (int j = 0; j < NH; j++) {
        float a = w[OFF_B2 + j];
        for (int i = 0; i < NH; i++) a += w[OFF_W2 + j * NH + i] * h1[i];
        a = a > 0.0f ? a : 0.0f;
        H2[s * NH + j] = a;
        y += w[OFF_W3 + j] * a;
    }
    Y[s] = y;
}

// per-sample output and hidden gradients of the loss mean((y - t)^2)
__global__ void __launch_bounds__(256)
k_mlp_bwd_rows(const float* __restrict__ p, const float* __restrict__ H1,
               const float* __restrict__ H2, const float* __restrict__ Y,
               const float* __restrict__ T, int64_t n, float* __restrict__ DY,
               float* __restrict__ DH2, float* __restrict__ DH1) {
    __shared__ float w2[NH * NH], w3[NH];
    for (int i = threadIdx.x; i < NH * NH; i += 256) w2[i] = p[OFF_W2 + i];
    for (int i = threadIdx.x; i < NH; i += 256) w3[i] = p[OFF_W3 + i];
    __syncthreads();
    int64_t s = blockIdx.x * 256ll + threadIdx.x;
    if (s >= n) return;
    float dy = 2.0f * (Y[s] - T[s]) / (float)n;
    DY[s] = dy;
    float dh2[NH];
    for (int j = 0; j < NH; j++) {
        dh2[j] = H2[s * NH + j] > 0.0f ? dy * w3[j] : 0.0f;
        DH2[s * NH + j] = dh2[j];
    }
    for (int i = 0; i < NH; i++) {
        float a = 0.0f;
        for (int j = 0; j < NH; j++) a += w2[j * NH + i] * dh2[j];
        DH1[s * NH + i] = H1[s * NH + i] > 0.0f ? a : 0.0f;
    }
}

// parameter gradients: one thread per parameter, a fixed-order sum over the
// batch (deterministic, no atomics)
__global__ void __launch_bounds__(256)
k_mlp_wgrad(const float* __restrict__ X, const float* __restrict__ H1,
            const float* __restrict__ H2, const float* __restrict__ DY,
            const float* __restrict__ DH2, const float* __restrict__ DH1, int64_t n,
            float* __restrict__ G) {
    int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= NPARAM) return;
    float acc = 0.0f;
    if (q < OFF_B1) {
        int j = q / NIN, i = q % NIN;
        for (int64_t s = 0; s < n; s++) acc += DH1[s * NH + j] * X[s * NIN + i];
    } else if (q < OFF_W2) {
        int j = q - OFF_B1;
        for (int64_t s = 0; s < n; s++) acc += DH1[s * NH + j];
    } else if (q < OFF_B2) {
        int j = (q - OFF_W2) / NH, i = (q - OFF_W2) % NH;
        for (int64_t s = 0; s < n; s++) acc += DH2[s * NH + j] * H1[s * NH + i];
    } else if (q < OFF_W3) {
        int j = q - OFF_B2;
        for (int64_t s = 0; s < n; s++) acc += DH2[s * NH + j];
    } else if (q < OFF_B3) {
        int j = q - OFF_W3;
        for (int64_t s = 0; s < n; s++) acc += DY[s] * H2[s * NH + j];
    } else {
        for (int64_t s = 0; s < n; s++) acc += DY[s];
    }
    G[q] = acc;
}

__global__ void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                           float* __restrict__ loss) {
    // one block: fixed-order sum (tree over the block, strided per thread)
    __shared__ float part[256];
    float a = 0.0f;
    for (int64_t s = threadIdx.x; s < n; s += 256) {
        float d = Y[s] - T[s];
        a += d * d;
    }
    part[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (float)n;
}

__global__ void k_mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
    int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= NPARAM) return;
    float gq = g[q];
    float mq = b1 * m[q] + (1.0f - b1) * gq;
    float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    float mh = mq / c1, vh = vq / c2;
    p[q] -= lr * mh / (sqrtf(vh) + eps);
}

// per-feature mean and standard deviation (one thread per feature)
__global__ void k_mlp_stats(const float* __restrict__ X, int64_t n, float* __restrict__ mean,
                            float* __restrict__ stdv) {
    int i = threadIdx.x;
    if (i >= NIN) return;
    double s = 0.0, s2 = 0.0;
    for (int64_t k = 0; k < n; k++) {
        double v = X[k * NIN + i];
        s += v;
        s2 += v * v;
    }
    double mu = n > 0 ? s / (double)n : 0.0;
    double var = n > 0 ? s2 / (double)n - mu * mu : 0.0;
    mean[i] = (float)mu;
    stdv[i] = var > 1e-12 ? (float)sqrt(var) : 1.0f;
}

__global__ void k_mlp_standardize(float* __restrict__ X, int64_t n, const float* __restrict__ mean,
                                  const float* __restrict__ stdv) {
    int64_t q = blockIdx.x * 256ll + threadIdx.x;
    if (q >= n * NIN) return;
    int i = (int)(q % NIN);
    X[q] = (X[q] - mean[i]) / stdv[i];
}

// ---------------------------------------------------------------------------
// node inference: bf16 weights and activations, fp32 accumulation
// ---------------------------------------------------------------------------

RS_DEV float bf16_round(float x) {
    // round to nearest even at 8 mantissa bits (finite inputs)
    uint32_t u = __float_as_uint(x);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return __uint_as_float(u & 0xffff0000u);
}

__global__ void __launch_bounds__(256)
k_mlp_infer(const float* __restrict__ model, int nv, const float* __restrict__ feat,
            float* __restrict__ out_ln_l) {
    __shared__ float w[NPARAM];
    __shared__ float mu[NIN], sd[NIN];
    const float* p = model + 2 * NIN;
    for (int i = threadIdx.x; i < NPARAM; i += 256) w[i] = bf16_round(p[i]);
    for (int i = threadIdx.x; i < NIN; i += 256) {
        mu[i] = model[i];
        sd[i] = model[NIN + i];
    }
    __syncthreads();
    int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    float x[NIN], h1[NH];
#pragma unroll
    for (int i = 0; i < NIN; i++) x[i] = bf16_round((feat[(int64_t)v * NIN + i] - mu[i]) / sd[i]);
    for (int j = 0; j < NH; j++) {
        float a = w[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < NIN; i++) a += w[OFF_W1 + j * NIN + i] * x[i];
        h1[j] = bf16_round(a > 0.0f ? a : 0.0f);
    }
    float y = w[OFF_B3];
    for (int j = 0; j < NH; j++) {
        float a = w[OFF_B2 + j];
        for (int i = 0; i < NH; i++) a += w[OFF_W2 + j * NH + i] * h1[i];
        y += w[OFF_W3 + j] * bf16_round(a > 0.0f ? a : 0.0f);
    }
    out_ln_l[v] = y;
}

int mlp_infer(const float* model_dev, int nv, const float* feat, float* out, hipStream_t st) {
    if (nv <= 0) return RS_OK;
    k_mlp_infer<<<(nv + 255) / 256, 256, 0, st>>>(model_dev, nv, feat, out);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

static int mlp_scratch(int64_t n, float** h1, float** h2, float** y, float** dy, float** dh2,
                       float** dh1, float** g, float** loss) {
    size_t b = 0;
    auto add = [&](size_t x) { b += arena_round(x); };
    add(4 * NH * n); add(4 * NH * n); add(4 * n); add(4 * n); add(4 * NH * n); add(4 * NH * n);
    add(4 * NPARAM); add(64);
    Arena* ar;
    RS_TRY(arena_call_begin(1u << AR_MLP));   // only the standalone proposer entry points get here
    RS_TRY(arena_reserve(AR_MLP, b, &ar));
    *h1 = take<float>(ar, NH * n);
    *h2 = take<float>(ar, NH * n);
    *y = take<float>(ar, n);
    *dy = take<float>(ar, n);
    *dh2 = take<float>(ar, NH * n);
    *dh1 = take<float>(ar, NH * n);
    *g = take<float>(ar, NPARAM);
    *loss = take<float>(ar, 16);
    return *loss ? RS_OK : RS_EINTERNAL;
}

static int mlp_grad_impl(const float* params, const float* X, const float* T, int64_t n,
                         float** g_out, float** loss_out, hipStream_t st) {
    float *h1, *h2, *y, *dy, *dh2, *dh1, *g, *loss;
    RS_TRY(mlp_scratch(n, &h1, &h2, &y, &dy, &dh2, &dh1, &g, &loss));
    unsigned gb = (unsigned)((n + 255) / 256);
    k_mlp_fwd<<<gb, 256, 0, st>>>(params, X, n, h1, h2, y);
    k_mlp_loss<<<1, 256, 0, st>>>(y, T, n, loss);
    k_mlp_bwd_rows<<<gb, 256, 0, st>>>(params, h1, h2, y, T, n, dy, dh2, dh1);
    k_mlp_wgrad<<<(NPARAM + 255) / 256, 256, 0, st>>>(X, h1, h2, dy, dh2, dh1, n, g);
    RS_HIP(hipGetLastError());
    *g_out = g;
    *loss_out = loss;
    return RS_OK;
}

}  // namespace rs

extern "C" {

int rs_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream) {
    if (!params || (n > 0 && (!X || !y)) || n < 0) return RS_EINVAL;
    if (n == 0) return RS_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *h1, *h2, *yy, *dy, *dh2, *dh1, *g, *loss;
    RS_TRY(rs::mlp_scratch(n, &h1, &h2, &yy, &dy, &dh2, &dh1, &g, &loss));
    rs::k_mlp_fwd<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(params, X, n, h1, h2, y);
    RS_HIP(hipGetLastError());
    RS_HIP(hipStreamSynchronize(st));
    return RS_OK;
}

int rs_mlp_grad(const float* params, const float* X, const float* T, int64_t n, float* grad,
                float* loss, void* stream) {
    if (!params || !X || !T || !grad || !loss || n <= 0) return RS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *g, *l;
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::mlp_grad_impl(params, X, T, n, &g, &l, st));
    RS_HIP(hipMemcpyAsync(grad, g, 4 * rs::NPARAM, hipMemcpyDeviceToDevice, st));
    RS_HIP(hipMemcpyAsync(loss, l, 4, hipMemcpyDeviceToDevice, st));
    RS_HIP(hipStreamSynchronize(st));
    return RS_OK;
}

int rs_mlp_train_step(float* params, float* m, float* v, int64_t step, const float* X,
                      const float* T, int64_t n, float lr, float* loss, void* stream) {
    if (!params || !m || !v || !X || !T || !loss || n <= 0 || step < 1 || !(lr > 0.0f))
        return RS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *g, *l;
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::mlp_grad_impl(params, X, T, n, &g, &l, st));
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    rs::k_mlp_adam<<<(rs::NPARAM + 255) / 256, 256, 0, st>>>(params, m, v, g, lr, b1, b2, 1e-8f,
                                                             c1, c2);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(loss, l, 4, hipMemcpyDeviceToDevice, st));
    return RS_OK;
}

int rs_mlp_standardize(float* X, int64_t n, float* mean, float* stdv, int compute, void* stream) {
    if (!X || !mean || !stdv || n < 0) return RS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (compute) rs::k_mlp_stats<<<1, 64, 0, st>>>(X, n, mean, stdv);
    if (n > 0)
        rs::k_mlp_standardize<<<(unsigned)((n * rs::NIN + 255) / 256), 256, 0, st>>>(X, n, mean,
                                                                                  stdv);
    RS_HIP(hipGetLastError());
    return RS_OK;
}

int rs_mlp_infer(const float* model, int64_t n, const float* feat, float* out, void* stream) {
    if (!model || n < 0 || (n > 0 && (!feat || !out))) return RS_EINVAL;
    RS_TRY(rs::mlp_infer(model, (int)n, feat, out, static_cast<hipStream_t>(stream)));
    RS_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    return RS_OK;
}

}  // extern "C"
