// Per-orbital MLP of the learned fsGW warm start: features, forward,
// backward and Adam, FP32 on the device.
//
// Network 3 -> 128 -> 128 -> 128 -> 1, SiLU (x * sigmoid(x)) after each hidden
// layer; inputs standardised with norm[0..2] (mean) and norm[3..5] (std), the
// output mapped to target units as y = norm[6] + norm[7] * out; the loss is
// the mean of ((y - t) / norm[7])^2.  Parameters are one flat vector: W1
// [128][3], b1, W2 [128][128], b2, W3 [128][128], b3, W4 [1][128], b4.
// Activations kept for the backward pass: act = [z1, a1, z2, a2, z3, a3],
// each [rows][128].  Every reduction runs in a fixed order (no atomics), so
// results are deterministic.
#include "internal.h"

#include <cmath>

namespace gwm {

namespace {

constexpr int NIN = 3, HID = 128;
constexpr long OFF_W1 = 0, OFF_B1 = OFF_W1 + HID * NIN, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
               OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * HID, OFF_W4 = OFF_B3 + HID, OFF_B4 = OFF_W4 + HID,
               NPARAM = OFF_B4 + 1;

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

// feat[p] = (eps_p, sum_{P,q} L[P,p,q]^2, eps_p - mu_mid); one block per orbital
__global__ void features_kernel(int nocc, int nmo, int naux, const double* __restrict__ eps,
                                const double* __restrict__ L, float* __restrict__ feat) {
    const int p = blockIdx.x;
    __shared__ double part[256];
    double s = 0.0;
    const long M2 = (long)nmo * nmo;
    for (long i = threadIdx.x; i < (long)naux * nmo; i += blockDim.x) {
        const long P = i / nmo, q = i - P * nmo;
        const double x = L[P * M2 + (long)p * nmo + q];
        s += x * x;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = 0.5 * (eps[nocc - 1] + eps[nocc]);
        feat[p * 3 + 0] = (float)eps[p];
        feat[p * 3 + 1] = (float)part[0];
        feat[p * 3 + 2] = (float)(eps[p] - mu);
    }
}

// z1 = W1 xhat + b1, a1 = silu(z1); one block (HID threads) per row
__global__ void layer1_kernel(int rows, const float* __restrict__ prm, const float* __restrict__ norm,
                              const float* __restrict__ x, float* __restrict__ z, float* __restrict__ a) {
    const int r = blockIdx.x, j = threadIdx.x;
    if (r >= rows) return;
    float s = prm[OFF_B1 + j];
#pragma unroll
    for (int k = 0; k < NIN; ++k) s += prm[OFF_W1 + j * NIN + k] * ((x[r * NIN + k] - norm[k]) / norm[3 + k]);
    z[(long)r * HID + j] = s;
    a[(long)r * HID + j] = silu(s);
}

// z = W ain + b, a = silu(z) for a HID x HID layer; one block per row
__global__ void hidden_kernel(int rows, const float* __restrict__ W, const float* __restrict__ b,
                              const float* __restrict__ ain, float* __restrict__ z, float* __restrict__ a) {
    const int r = blockIdx.x, j = threadIdx.x;
    if (r >= rows) return;
    __shared__ float in[HID];
    in[j] = ain[(long)r * HID + j];
    __syncthreads();
    float s = b[j];
    for (int k = 0; k < HID; ++k) s += W[j * HID + k] * in[k];
    z[(long)r * HID + j] = s;
    a[(long)r * HID + j] = silu(s);
}

// y = norm[6] + norm[7] * (W4 a3 + b4); one wave per row
__global__ void out_kernel(int rows, const float* __restrict__ prm, const float* __restrict__ norm,
                           const float* __restrict__ a3, float* __restrict__ y) {
    const long r = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;
    float s = prm[OFF_W4 + lane] * a3[r * HID + lane] + prm[OFF_W4 + 64 + lane] * a3[r * HID + 64 + lane];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[r] = norm[6] + norm[7] * (s + prm[OFF_B4]);
}

// d_out[r] = (2/rows) (y - t) / std_t ;  dz3[r][j] = d_out[r] W4[j] silu'(z3[r][j])
__global__ void dout_kernel(int rows, const float* __restrict__ prm, const float* __restrict__ norm,
                            const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ z3,
                            float* __restrict__ dout, float* __restrict__ dz3) {
    const int r = blockIdx.x, j = threadIdx.x;
    if (r >= rows) return;
    const float d = 2.0f / rows * (y[r] - t[r]) / norm[7];
    if (j == 0) dout[r] = d;
    dz3[(long)r * HID + j] = d * prm[OFF_W4 + j] * dsilu(z3[(long)r * HID + j]);
}

// gW[j][k] = sum_r dz[r][j] ain(r, k), gb[j] = sum_r dz[r][j]; one block (nin threads) per j.
// ain(r, k) is act[r*nin + k], or the standardised input when xin is set (layer 1).
__global__ void wgrad_kernel(int rows, int nout, int nin, long ldz, const float* __restrict__ dz,
                             const float* __restrict__ ain, const float* __restrict__ xin,
                             const float* __restrict__ norm, float* __restrict__ gW, float* __restrict__ gb) {
    const int j = blockIdx.x, k = threadIdx.x;
    if (j >= nout) return;
    float s = 0.0f, sb = 0.0f;
    for (int r = 0; r < rows; ++r) {
        const float d = dz[(long)r * ldz + j];
        float av;
        if (xin) av = k < nin ? (xin[r * NIN + k] - norm[k]) / norm[3 + k] : 0.0f;
        else av = ain[(long)r * nin + k];
        s += d * av;
        sb += d;
    }
    if (k < nin) gW[j * nin + k] = s;
    if (k == 0) gb[j] = sb;
}

// dzp[r][k] = (sum_j dz[r][j] W[j][k]) silu'(zp[r][k]) for a HID x HID layer; one block per row
__global__ void dback_kernel(int rows, const float* __restrict__ W, const float* __restrict__ dz,
                             const float* __restrict__ zp, float* __restrict__ dzp) {
    const int r = blockIdx.x, k = threadIdx.x;
    if (r >= rows) return;
    __shared__ float d[HID];
    d[k] = dz[(long)r * HID + k];
    __syncthreads();
    float s = 0.0f;
    for (int j = 0; j < HID; ++j) s += d[j] * W[j * HID + k];
    dzp[(long)r * HID + k] = s * dsilu(zp[(long)r * HID + k]);
}

// loss = mean(((y - t) / std_t)^2), one block
__global__ void loss_kernel(int rows, const float* __restrict__ norm, const float* __restrict__ y,
                            const float* __restrict__ t, float* __restrict__ loss) {
    __shared__ float part[256];
    float s = 0.0f;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const float e = (y[r] - t[r]) / norm[7];
        s += e * e;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = part[0] / rows;
}

__global__ void adam_kernel(long n, float lr, float b1, float b2, float eps, float c1, float c2,
                            float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// norm = (mean of the three feature columns, their standard deviations, mean
// and standard deviation of the targets) over rows: one block, FP64 partial
// sums per thread over a fixed row stride, then a fixed-order tree; two
// passes (means, then squared deviations); deviations floored at 1e-12.
__global__ void norm_kernel(int rows, const float* __restrict__ x, const float* __restrict__ t,
                            float* __restrict__ norm) {
    __shared__ double sh[4][256];
    __shared__ double mean[4];
    const int tid = threadIdx.x;
    for (int pass = 0; pass < 2; ++pass) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = tid; r < rows; r += 256) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double v = c < 3 ? (double)x[(long)r * 3 + c] : (double)t[r];
                const double d = pass ? v - mean[c] : v;
                s[c] += pass ? d * d : d;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[c][tid] = s[c];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w)
#pragma unroll
                for (int c = 0; c < 4; ++c) sh[c][tid] += sh[c][tid + w];
            __syncthreads();
        }
        if (tid < 4) {
            const double v = sh[tid][0] / rows;
            if (pass == 0) {
                mean[tid] = v;
                norm[tid < 3 ? tid : 6] = (float)v;
            } else {
                norm[tid < 3 ? 3 + tid : 7] = (float)fmax(sqrt(v), 1e-12);
            }
        }
        __syncthreads();
    }
}

// t[p] = F[p][p] - eps[p]
__global__ void target_kernel(int nmo, const double* __restrict__ F, const double* __restrict__ eps,
                              float* __restrict__ t) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nmo) t[p] = (float)(F[(long)p * nmo + p] - eps[p]);
}

// F0 = diag(eps + y)
__global__ void warm_start_kernel(int nmo, const double* __restrict__ eps, const float* __restrict__ y,
                                  double* __restrict__ F0) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nmo * nmo) return;
    const long p = i / nmo, q = i - p * nmo;
    F0[i] = p == q ? eps[p] + (double)y[p] : 0.0;
}

}  // namespace

long mlp_param_count() { return NPARAM; }

gw_status mlp_norm(Handle* h, int rows, const float* x, const float* t, float* norm) {
    hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(256), 0, h->stream, rows, x, t, norm);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status mlp_target(Handle* h, int nmo, const double* F, const double* eps, float* t) {
    hipLaunchKernelGGL(target_kernel, dim3((unsigned)((nmo + 255) / 256)), dim3(256), 0, h->stream, nmo, F, eps, t);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status mlp_warm_start(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* L,
                         const float* prm, const float* norm, double* F0) {
    const int nmo = nocc + nvir;
    float* buf = (float*)ws_get(h, WS_FS6, sizeof(float) * 4L * nmo);
    if (!buf) return GW_ENOMEM;
    float *feat = buf, *y = buf + 3L * nmo;
    GW_TRY(mlp_features(h, nocc, nvir, naux, eps, L, feat));
    GW_TRY(mlp_forward(h, nmo, prm, norm, feat, nullptr, y));
    const long n = (long)nmo * nmo;
    hipLaunchKernelGGL(warm_start_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, nmo, eps, y, F0);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status mlp_features(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* L, float* feat) {
    const int nmo = nocc + nvir;
    hipLaunchKernelGGL(features_kernel, dim3(nmo), dim3(256), 0, h->stream, nocc, nmo, naux, eps, L, feat);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status mlp_forward(Handle* h, int rows, const float* prm, const float* norm, const float* x, float* act, float* y) {
    if (!act) {
        act = (float*)ws_get(h, WS_MISC, sizeof(float) * 6L * rows * HID);
        if (!act) return GW_ENOMEM;
    }
    const long st = (long)rows * HID;
    float *z1 = act, *a1 = act + st, *z2 = act + 2 * st, *a2 = act + 3 * st, *z3 = act + 4 * st, *a3 = act + 5 * st;
    hipLaunchKernelGGL(layer1_kernel, dim3(rows), dim3(HID), 0, h->stream, rows, prm, norm, x, z1, a1);
    hipLaunchKernelGGL(hidden_kernel, dim3(rows), dim3(HID), 0, h->stream, rows, prm + OFF_W2, prm + OFF_B2, a1, z2,
                       a2);
    hipLaunchKernelGGL(hidden_kernel, dim3(rows), dim3(HID), 0, h->stream, rows, prm + OFF_W3, prm + OFF_B3, a2, z3,
                       a3);
    hipLaunchKernelGGL(out_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, h->stream, rows, prm, norm, a3, y);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status mlp_backward(Handle* h, int rows, const float* prm, const float* norm, const float* x, const float* act,
                       const float* y, const float* t, float* grad, float* loss) {
    const long st = (long)rows * HID;
    const float *z1 = act, *a1 = act + st, *z2 = act + 2 * st, *a2 = act + 3 * st, *z3 = act + 4 * st,
                *a3 = act + 5 * st;
    float* buf = (float*)ws_get(h, WS_FS7, sizeof(float) * (2 * st + rows));
    if (!buf) return GW_ENOMEM;
    float *dA = buf, *dB = buf + st, *dout = buf + 2 * st;
    hipLaunchKernelGGL(dout_kernel, dim3(rows), dim3(HID), 0, h->stream, rows, prm, norm, y, t, z3, dout, dA);
    // output layer: gW4[k] = sum_r dout[r] a3[r][k], gb4 = sum_r dout[r]
    hipLaunchKernelGGL(wgrad_kernel, dim3(1), dim3(HID), 0, h->stream, rows, 1, HID, 1L, dout, a3,
                       (const float*)nullptr, norm, grad + OFF_W4, grad + OFF_B4);
    // layer 3 (dA = dz3)
    hipLaunchKernelGGL(wgrad_kernel, dim3(HID), dim3(HID), 0, h->stream, rows, HID, HID, (long)HID, dA, a2,
                       (const float*)nullptr, norm, grad + OFF_W3, grad + OFF_B3);
    hipLaunchKernelGGL(dback_kernel, dim3(rows), dim3(HID), 0, h->stream, rows, prm + OFF_W3, dA, z2, dB);
    // layer 2 (dB = dz2)
    hipLaunchKernelGGL(wgrad_kernel, dim3(HID), dim3(HID), 0, h->stream, rows, HID, HID, (long)HID, dB, a1,
                       (const float*)nullptr, norm, grad + OFF_W2, grad + OFF_B2);
    hipLaunchKernelGGL(dback_kernel, dim3(rows), dim3(HID), 0, h->stream, rows, prm + OFF_W2, dB, z1, dA);
    // layer 1 (dA = dz1), inputs standardised on the fly
    hipLaunchKernelGGL(wgrad_kernel, dim3(HID), dim3(64), 0, h->stream, rows, HID, NIN, (long)HID, dA,
                       (const float*)nullptr, x, norm, grad + OFF_W1, grad + OFF_B1);
    if (loss) hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, h->stream, rows, norm, y, t, loss);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status mlp_adam(Handle* h, int step, float lr, float b1, float b2, float eps, float* prm, const float* grad,
                   float* m, float* v) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, h->stream, NPARAM, lr, b1,
                       b2, eps, c1, c2, prm, grad, m, v);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

}  // namespace gwm
