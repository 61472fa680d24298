// Cost model of the scheduler: a perceptron with two hidden ReLU layers of
// 64 units, FP32, trained on the mean squared error with Adam, entirely on
// the device.
//
//   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 w3 + b3
//   L  = mean_i (y_i - t_i)^2
//
// Parameters: one flat FP32 vector W1[F][64], b1[64], W2[64][64], b2[64],
// w3[64], b3[1].
//
// k_mlp_sample: one thread per sample; weights staged in LDS; computes the
//   forward pass and, when training, the per-sample back-propagated terms
//   dz1, dz2 (64 each) and dy, stored for the reduction.
// k_mlp_reduce: one thread per parameter; sums its gradient over the batch in
//   a fixed order (deterministic), e.g. dL/dW2[a][j] = sum_i h1[i][a] dz2[i][j].
// k_mlp_adam:   one thread per parameter; Adam step k.
// k_standardize, k_affine_base: the cost model's input and output scaling
//   around the network, (x - mu) * isd per feature and y * sd + mu, plus the
//   raw base feature (the network predicts the correction to it).
#include <cmath>
#include <vector>

#include "epi_internal.h"

namespace epi {

namespace {

constexpr int kH = kMlpHidden;

__host__ __device__ inline int64_t n_params_of(int F) { return (int64_t)F * kH + kH + kH * kH + kH + kH + 1; }

__global__ __launch_bounds__(256) void k_mlp_sample(const float *__restrict__ p, int F, const float *__restrict__ X,
                                                    const float *__restrict__ t, int64_t B, float *__restrict__ y,
                                                    float *__restrict__ h1s, float *__restrict__ dz1s,
                                                    float *__restrict__ dz2s, float *__restrict__ h2s,
                                                    float *__restrict__ dys, float *__restrict__ sqerr) {
    extern __shared__ float w[];
    const int64_t np = n_params_of(F);
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) w[i] = p[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const float *W1 = w, *b1 = w + F * kH, *W2 = b1 + kH, *b2 = W2 + kH * kH, *w3 = b2 + kH, *b3 = w3 + kH;
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) h1[j] = b1[j];
    for (int f = 0; f < F; ++f) {
        const float x = X[s * F + f];
#pragma unroll
        for (int j = 0; j < kH; ++j) h1[j] = fmaf(x, W1[f * kH + j], h1[j]);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) h1[j] = h1[j] > 0.f ? h1[j] : 0.f;  // z1 > 0 <=> h1 > 0
    float out = b3[0];
    float z2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) z2[j] = b2[j];
    for (int a = 0; a < kH; ++a) {
        const float v = h1[a];
#pragma unroll
        for (int j = 0; j < kH; ++j) z2[j] = fmaf(v, W2[a * kH + j], z2[j]);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) out = fmaf(z2[j] > 0.f ? z2[j] : 0.f, w3[j], out);
    y[s] = out;
    if (!t) return;
    const float r = out - t[s];
    sqerr[s] = r * r;
    const float dy = 2.f * r / (float)B;
    dys[s] = dy;
    // dz2 = dy * w3 * [z2 > 0];  dz1 = (dz2 W2^T) * [z1 > 0]
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        const float h2 = z2[j] > 0.f ? z2[j] : 0.f;
        h2s[s * kH + j] = h2;
        z2[j] = z2[j] > 0.f ? dy * w3[j] : 0.f;  // now dz2
        dz2s[s * kH + j] = z2[j];
    }
    for (int a = 0; a < kH; ++a) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc = fmaf(z2[j], W2[a * kH + j], acc);
        h1s[s * kH + a] = h1[a];
        dz1s[s * kH + a] = h1[a] > 0.f ? acc : 0.f;
    }
}

// gradient of one parameter, summed over the batch in sample order
__global__ __launch_bounds__(256) void k_mlp_reduce(int F, const float *__restrict__ X, int64_t B,
                                                    const float *__restrict__ h1s, const float *__restrict__ dz1s,
                                                    const float *__restrict__ dz2s, const float *__restrict__ h2s,
                                                    const float *__restrict__ dys, float *__restrict__ g) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = n_params_of(F);
    if (q >= np) return;
    float acc = 0.f;
    int64_t o = q;
    if (o < (int64_t)F * kH) {  // W1[f][j]: x_f dz1_j
        const int f = (int)(o / kH), j = (int)(o % kH);
        for (int64_t i = 0; i < B; ++i) acc = fmaf(X[i * F + f], dz1s[i * kH + j], acc);
    } else if ((o -= (int64_t)F * kH) < kH) {  // b1
        for (int64_t i = 0; i < B; ++i) acc += dz1s[i * kH + o];
    } else if ((o -= kH) < kH * kH) {  // W2[a][j]: h1_a dz2_j
        const int a = (int)(o / kH), j = (int)(o % kH);
        for (int64_t i = 0; i < B; ++i) acc = fmaf(h1s[i * kH + a], dz2s[i * kH + j], acc);
    } else if ((o -= kH * kH) < kH) {  // b2
        for (int64_t i = 0; i < B; ++i) acc += dz2s[i * kH + o];
    } else if ((o -= kH) < kH) {  // w3[j]: h2_j dy
        for (int64_t i = 0; i < B; ++i) acc = fmaf(h2s[i * kH + o], dys[i], acc);
    } else {  // b3
        for (int64_t i = 0; i < B; ++i) acc += dys[i];
    }
    g[q] = acc;
}

__global__ void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

__global__ void k_standardize(float *__restrict__ X, int64_t n, int F, const float *__restrict__ norm) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int f = (int)(q % F);
    X[q] = (X[q] - norm[f]) * norm[F + f];
}

// y = y * sd + mu + x_base, where x_base is the raw value of input feature
// `base` of the sample (recovered from the standardised Xs: x = x' / isd + mu;
// a constant feature, isd = 0, is its mean); base < 0: no base term.
__global__ void k_affine_base(float *__restrict__ y, int64_t n, float sd, float mu, const float *__restrict__ Xs,
                              int F, const float *__restrict__ norm, int base) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    float b = 0.f;
    if (base >= 0) {
        const float isd = norm[F + base], m = norm[base];
        b = isd > 0.f ? Xs[q * F + base] / isd + m : m;
    }
    y[q] = fmaf(y[q], sd, mu) + b;
}

}  // namespace

int64_t mlp_n_params(int F) { return n_params_of(F); }

hipError_t mlp_set_scaling(Mlp &net, const float *x_mu, const float *x_isd, float y_mu, float y_sd) {
    net.x_mu.assign(x_mu, x_mu + net.F);
    net.x_isd.assign(x_isd, x_isd + net.F);
    net.y_mu = y_mu;
    net.y_sd = y_sd;
    std::vector<float> h(net.x_mu);
    h.insert(h.end(), net.x_isd.begin(), net.x_isd.end());
    hipError_t e;
    if (!net.norm.p && (e = net.norm.alloc(sizeof(float) * 2 * net.F)) != hipSuccess) return e;
    return hipMemcpy(net.norm.p, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice);
}

hipError_t costmodel_predict_device(Mlp &net, float *dX, int64_t B, float *dy, hipStream_t st) {
    if (B == 0) return hipSuccess;
    const int64_t n = B * net.F;
    k_standardize<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(dX, n, net.F, net.norm.as<float>());
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = mlp_forward_device(net, dX, B, dy, st)) != hipSuccess) return e;
    k_affine_base<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(dy, B, net.y_sd, net.y_mu, dX, net.F,
                                                                net.norm.as<float>(),
                                                                net.F > kBaseFeature ? kBaseFeature : -1);
    return hipGetLastError();
}

hipError_t mlp_forward_device(Mlp &net, const float *dX, int64_t B, float *dy, hipStream_t st) {
    if (B == 0) return hipSuccess;
    const size_t lds = sizeof(float) * (size_t)n_params_of(net.F);
    k_mlp_sample<<<(unsigned)((B + 255) / 256), 256, lds, st>>>(net.p.as<float>(), net.F, dX, nullptr, B, dy, nullptr,
                                                               nullptr, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t mlp_grad_device(Mlp &net, const float *dX, const float *dt, int64_t B, float *dg, float *loss,
                           hipStream_t st) {
    hipError_t e;
    if ((size_t)B > net.cap) {
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if ((e = net.act.alloc(sizeof(float) * (size_t)B * (4 * kH + 3))) != hipSuccess) return e;
        net.cap = (size_t)B;
    }
    float *base = net.act.as<float>();
    float *h1s = base, *dz1s = h1s + B * kH, *dz2s = dz1s + B * kH, *h2s = dz2s + B * kH;
    float *dys = h2s + B * kH, *ys = dys + B, *sq = ys + B;
    const size_t lds = sizeof(float) * (size_t)n_params_of(net.F);
    k_mlp_sample<<<(unsigned)((B + 255) / 256), 256, lds, st>>>(net.p.as<float>(), net.F, dX, dt, B, ys, h1s, dz1s,
                                                               dz2s, h2s, dys, sq);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t np = n_params_of(net.F);
    k_mlp_reduce<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(net.F, dX, B, h1s, dz1s, dz2s, h2s, dys, dg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (loss) {
        std::vector<float> h(B);
        if ((e = hipMemcpyAsync(h.data(), sq, sizeof(float) * B, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        double acc = 0;
        for (float x : h) acc += x;
        *loss = (float)(acc / (double)B);
    }
    return hipSuccess;
}

hipError_t mlp_adam_device(Mlp &net, const float *dg, hipStream_t st) {
    const int64_t np = n_params_of(net.F);
    net.step += 1;
    const float c1 = 1.f - std::pow(net.b1, (float)net.step);
    const float c2 = 1.f - std::pow(net.b2, (float)net.step);
    k_mlp_adam<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(net.p.as<float>(), dg, net.m.as<float>(),
                                                              net.v.as<float>(), np, net.lr, net.b1, net.b2, net.eps,
                                                              c1, c2);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014): counter-based, used only for the initial weights.
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

hipError_t mlp_init(Mlp &net, int F, uint64_t seed) {
    net.F = F;
    net.step = 0;
    const int64_t np = n_params_of(F);
    std::vector<float> h(np, 0.f);
    // uniform(-s, s) with s = sqrt(6 / fan_in) for weights (He-uniform), zero biases
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double s = std::sqrt(6.0 / fan_in);
        for (int64_t i = 0; i < count; ++i) {
            const double u = (double)(splitmix64(seed * 0x100000001B3ull + (uint64_t)(off + i)) >> 11) * 0x1.0p-53;
            h[off + i] = (float)((2.0 * u - 1.0) * s);
        }
    };
    fill(0, (int64_t)F * kH, F);
    fill((int64_t)F * kH + kH, kH * kH, kH);
    fill((int64_t)F * kH + kH + kH * kH + kH, kH, kH);
    hipError_t e;
    if ((e = net.p.alloc(sizeof(float) * np)) != hipSuccess) return e;
    if ((e = net.m.alloc(sizeof(float) * np)) != hipSuccess) return e;
    if ((e = net.v.alloc(sizeof(float) * np)) != hipSuccess) return e;
    if ((e = net.g.alloc(sizeof(float) * np)) != hipSuccess) return e;
    if ((e = hipMemcpy(net.p.p, h.data(), sizeof(float) * np, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemset(net.m.p, 0, sizeof(float) * np)) != hipSuccess) return e;
    if ((e = hipMemset(net.v.p, 0, sizeof(float) * np)) != hipSuccess) return e;
    net.norm.reset();
    const std::vector<float> zero(F, 0.f), one(F, 1.f);
    return mlp_set_scaling(net, zero.data(), one.data(), 0.f, 1.f);
}

}  // namespace epi
