// The learned l(t) surrogate of lbcap: an MLP 19 -> 256 -> 256 -> 256 -> 64
// with GELU activations, trained by mean-squared error and Adam, all on the
// device in FP32.
//
// Every dense product (forward, input gradient, weight gradient) runs through
// one MFMA kernel: 64 x 64 output tiles per workgroup of four wavefronts, each
// wavefront a 32 x 32 block of 2 x 2 v_mfma_f32_16x16x4f32 tiles, K staged
// through LDS 16 at a time.  Operand strides are free, so the transposed
// products of the backward pass read the stored activations and weights in
// place.  Bias, GELU and the GELU derivative are fused into the epilogue.
// Reductions (bias gradients, the loss) are sequential per output element or
// a fixed tree, so a training run is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbcap.h"
#include "lb_internal.h"

namespace {

constexpr int NLAYER = 4;
constexpr int DIMS[NLAYER + 1] = {19, 256, 256, 256, 64};
constexpr int WMAX = 256;               // widest layer

typedef float f4 __attribute__((ext_vector_type(4)));

enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

// C(m, n) = sum_k A(m, k) B(k, n) over an M x N x K problem, with
// A(m, k) = A[m sam + k sak] and B(k, n) = B[k sbk + n sbn]; one of each pair
// of strides is 1.  Epilogues:
//   EPI_STORE      C = acc
//   EPI_BIAS       C = acc + bias[n]
//   EPI_BIAS_GELU  C = z = acc + bias[n], H = gelu(z)      (H has C's layout)
//   EPI_GELU_BWD   C = acc * gelu'(Z)                        (Z has C's layout)
struct GemmArgs {
    int M, N, K;
    const float* A;
    long sam, sak;
    const float* B;
    long sbk, sbn;
    float* C;
    int ldc;
    const float* bias;
    float* H;
    const float* Z;
};

constexpr int BM = 64, BN = 64, BK = 16, PADL = 4;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

template <int EPI>
__global__ void __launch_bounds__(256) mlp_gemm(GemmArgs g) {
    __shared__ float As[BK][BM + PADL];   // k-major: a wavefront reads 16 consecutive m
    __shared__ float Bs[BK][BN + PADL];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = t + 256 * r;
            int m, k;
            if (g.sak == 1) { m = e >> 4; k = e & 15; } else { m = e & 63; k = e >> 6; }
            const int gm = m0 + m, gk = k0 + k;
            As[k][m] = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : 0.f;
            int n, kb;
            if (g.sbn == 1) { n = e & 63; kb = e >> 6; } else { n = e >> 4; kb = e & 15; }
            const int gn = n0 + n, gkb = k0 + kb;
            Bs[kb][n] = (gn < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gn * g.sbn] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kk + lk][wm + 16 * i + lr];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk + lk][wn + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // 16 x 16 result tile: lane holds rows 4 (lane / 16) + v, column lane % 16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm + 16 * i + 4 * lk + v;
                const int n = n0 + wn + 16 * j + lr;
                if (m >= g.M || n >= g.N) continue;
                const long o = (long)m * g.ldc + n;
                const float x = acc[i][j][v];
                if (EPI == EPI_STORE) {
                    g.C[o] = x;
                } else if (EPI == EPI_BIAS) {
                    g.C[o] = x + g.bias[n];
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = x + g.bias[n];
                    g.C[o] = z;
                    g.H[o] = gelu(z);
                } else {
                    g.C[o] = x * gelu_grad(g.Z[o]);
                }
            }
}

// db[j] = sum over rows of dZ[r][j], rows in order.
__global__ void mlp_bias_grad(const float* __restrict__ dZ, int rows, int cols, float* __restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += dZ[(long)r * cols + j];
    db[j] = s;
}

// Mean-squared error over rows x cols: dOut = 2 (out - y) / (rows cols) and
// loss = mean (out - y)^2, by one workgroup with a fixed reduction tree.
__global__ void __launch_bounds__(256) mlp_mse(const float* __restrict__ out, const float* __restrict__ y,
                                               long count, float* __restrict__ dout, float* __restrict__ loss) {
    __shared__ float red[256];
    const int t = threadIdx.x;
    const float inv = 1.f / (float)count;
    float s = 0.f;
    for (long e = t; e < count; e += 256) {
        const float d = out[e] - y[e];
        dout[e] = 2.f * d * inv;
        s += d * d;
    }
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) *loss = red[0] * inv;
}

// Adam (Kingma & Ba 2015, Algorithm 1); bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                         float* __restrict__ v, long count, float lr, float b1, float b2, float eps, float bc1,
                         float bc2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Rows idx[r] of X (cols_x wide) and Y (cols_y wide) into Xb, Yb.
__global__ void mlp_gather(const float* __restrict__ X, const float* __restrict__ Y, const int* __restrict__ idx,
                           int rows, int cols_x, int cols_y, float* __restrict__ Xb, float* __restrict__ Yb) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    const long src = idx[r];
    for (int c = threadIdx.x; c < cols_x; c += blockDim.x) Xb[(long)r * cols_x + c] = X[src * cols_x + c];
    for (int c = threadIdx.x; c < cols_y; c += blockDim.x) Yb[(long)r * cols_y + c] = Y[src * cols_y + c];
}

// ---- allocation-free inference scratch ------------------------------------------
// Activations of mlp_predict_device_noalloc: one buffer for the pre-activations
// the forward pass writes but inference does not read, and two that the hidden
// activations alternate between, each MLP_NOALLOC_MAX_ROWS x 256 floats
// (3 MiB in all).  Every GPU that runs the library holds its own copy until
// the process ends; host code addresses it only through the pointer that
// hipGetSymbolAddress returned for that GPU (noalloc_scratch below).
constexpr int SCRATCH_BUFS = 3;
constexpr long SCRATCH_BUF = (long)MLP_NOALLOC_MAX_ROWS * WMAX;
static __device__ __align__(256) float scratch[SCRATCH_BUFS * SCRATCH_BUF];

// ---- host side -----------------------------------------------------------------

long param_count() {
    long n = 0;
    for (int l = 0; l < NLAYER; ++l) n += (long)DIMS[l + 1] * DIMS[l] + DIMS[l + 1];
    return n;
}

long w_off(int l) {
    long n = 0;
    for (int i = 0; i < l; ++i) n += (long)DIMS[i + 1] * DIMS[i] + DIMS[i + 1];
    return n;
}
long b_off(int l) { return w_off(l) + (long)DIMS[l + 1] * DIMS[l]; }

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

double uniform01(uint64_t seed, uint64_t i) {
    return (double)(splitmix64(seed * 0x100000001B3ull + i) >> 11) * (1.0 / 9007199254740992.0);
}

#define MLP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return lbk::set_error(LB_EDEVICE, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

}  // namespace

struct mlp_net {
    int device = -1;           // the GPU the parameters live on
    hipStream_t stream = nullptr;
    float* P = nullptr;        // parameters, mlp_get_params layout
    float* G = nullptr;        // gradients, same layout
    float* Mo = nullptr;       // Adam first moments
    float* Vo = nullptr;       // Adam second moments
    long adam_t = 0;           // Adam steps taken
    int cap = 0;               // rows the activation buffers hold
    float* act[NLAYER] = {};   // layer inputs: act[0] = X, act[l] = gelu(z[l-1])
    float* z[NLAYER] = {};     // pre-activations; z[3] is the output
    float* d0 = nullptr;       // gradient buffers (ping-pong), cap x WMAX
    float* d1 = nullptr;
    float* yb = nullptr;       // targets of the current rows
    float* loss = nullptr;     // device scalars, one per minibatch
    int loss_cap = 0;
    float* Xall = nullptr;     // training set on the device
    float* Yall = nullptr;
    int* idx = nullptr;
    long data_cap = 0;
};

namespace {

void free_rows(mlp_net* n) {
    for (int l = 0; l < NLAYER; ++l) {
        (void)hipFree(n->act[l]);
        (void)hipFree(n->z[l]);
        n->act[l] = n->z[l] = nullptr;
    }
    (void)hipFree(n->d0);
    (void)hipFree(n->d1);
    (void)hipFree(n->yb);
    n->d0 = n->d1 = n->yb = nullptr;
    n->cap = 0;
}

lb_status ensure_rows(mlp_net* n, int rows) {
    if (rows <= n->cap) return LB_OK;
    MLP_TRY(hipStreamSynchronize(n->stream));
    free_rows(n);
    for (int l = 0; l < NLAYER; ++l) {
        MLP_TRY(hipMalloc(&n->act[l], sizeof(float) * (size_t)rows * DIMS[l]));
        MLP_TRY(hipMalloc(&n->z[l], sizeof(float) * (size_t)rows * DIMS[l + 1]));
    }
    MLP_TRY(hipMalloc(&n->d0, sizeof(float) * (size_t)rows * WMAX));
    MLP_TRY(hipMalloc(&n->d1, sizeof(float) * (size_t)rows * WMAX));
    MLP_TRY(hipMalloc(&n->yb, sizeof(float) * (size_t)rows * DIMS[NLAYER]));
    n->cap = rows;
    return LB_OK;
}

template <int EPI>
lb_status gemm(hipStream_t s, const GemmArgs& g) {
    if (g.M <= 0 || g.N <= 0) return LB_OK;
    dim3 grid((g.M + BM - 1) / BM, (g.N + BN - 1) / BN);
    hipLaunchKernelGGL(mlp_gemm<EPI>, grid, dim3(256), 0, s, g);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

// Forward pass of `rows` rows with parameters P on stream s: layer l reads
// in[l] and writes its pre-activation to z[l] and (hidden layers) its GELU to
// in[l + 1]; z[NLAYER-1] receives the output.
lb_status forward_bufs(hipStream_t s, const float* P, int rows, const float* const (&in)[NLAYER],
                       float* const (&z)[NLAYER]) {
    for (int l = 0; l < NLAYER; ++l) {
        const int ni = DIMS[l], no = DIMS[l + 1];
        GemmArgs g{};
        g.M = rows;
        g.N = no;
        g.K = ni;
        g.A = in[l];
        g.sam = ni;
        g.sak = 1;
        g.B = P + w_off(l);   // B(k, j) = W[j][k]
        g.sbk = 1;
        g.sbn = ni;
        g.C = z[l];
        g.ldc = no;
        g.bias = P + b_off(l);
        lb_status st;
        if (l + 1 < NLAYER) {
            g.H = const_cast<float*>(in[l + 1]);
            st = gemm<EPI_BIAS_GELU>(s, g);
        } else {
            st = gemm<EPI_BIAS>(s, g);
        }
        if (st) return st;
    }
    return LB_OK;
}

// Forward pass of `rows` rows of act[0]; output in z[NLAYER-1].
lb_status forward(mlp_net* n, int rows) {
    const float* const in[NLAYER] = {n->act[0], n->act[1], n->act[2], n->act[3]};
    float* const z[NLAYER] = {n->z[0], n->z[1], n->z[2], n->z[3]};
    return forward_bufs(n->stream, n->P, rows, in, z);
}

// Device address of this GPU's copy of `scratch`, resolved once per device
// (with that device current) by hipGetSymbolAddress: the array's name in host
// code is a host-side stand-in, not a device address.
std::mutex g_scratch_mu;
std::map<int, float*> g_scratch_ptr;

lb_status noalloc_scratch(int device, float** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return LB_OK;
    }
    int cur = -1;
    MLP_TRY(hipGetDevice(&cur));
    if (cur != device) return lbk::set_error(LB_ESTATE, "the network's device is not the current device");
    void* p = nullptr;
    MLP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = (float*)p;
    *out = (float*)p;
    return LB_OK;
}

// Backward pass from dOut (in d0, rows x 64) into G.
lb_status backward(mlp_net* n, int rows) {
    float* dz = n->d0;
    float* dn = n->d1;
    for (int l = NLAYER - 1; l >= 0; --l) {
        const int in = DIMS[l], out = DIMS[l + 1];
        // dW[o][i] = sum_r dz[r][o] act[r][i]
        GemmArgs gw{};
        gw.M = out;
        gw.N = in;
        gw.K = rows;
        gw.A = dz;
        gw.sam = 1;
        gw.sak = out;
        gw.B = n->act[l];
        gw.sbk = in;
        gw.sbn = 1;
        gw.C = n->G + w_off(l);
        gw.ldc = in;
        if (lb_status st = gemm<EPI_STORE>(n->stream, gw)) return st;
        hipLaunchKernelGGL(mlp_bias_grad, dim3((out + 255) / 256), dim3(256), 0, n->stream, dz, rows, out,
                           n->G + b_off(l));
        MLP_TRY(hipGetLastError());
        if (l == 0) break;
        // d act[r][i] = sum_o dz[r][o] W[o][i], times gelu'(z[l-1][r][i])
        GemmArgs gx{};
        gx.M = rows;
        gx.N = in;
        gx.K = out;
        gx.A = dz;
        gx.sam = out;
        gx.sak = 1;
        gx.B = n->P + w_off(l);
        gx.sbk = in;
        gx.sbn = 1;
        gx.C = dn;
        gx.ldc = in;
        gx.Z = n->z[l - 1];
        if (lb_status st = gemm<EPI_GELU_BWD>(n->stream, gx)) return st;
        std::swap(dz, dn);
    }
    return LB_OK;
}

lb_status mse(mlp_net* n, int rows, float* loss_slot) {
    hipLaunchKernelGGL(mlp_mse, dim3(1), dim3(256), 0, n->stream, n->z[NLAYER - 1], n->yb,
                       (long)rows * DIMS[NLAYER], n->d0, loss_slot);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

lb_status ensure_loss(mlp_net* n, int count) {
    if (count <= n->loss_cap) return LB_OK;
    MLP_TRY(hipStreamSynchronize(n->stream));
    (void)hipFree(n->loss);
    n->loss = nullptr;
    MLP_TRY(hipMalloc(&n->loss, sizeof(float) * (size_t)count));
    n->loss_cap = count;
    return LB_OK;
}

lb_status check_net(const mlp_net* n) {
    if (!n) return lbk::set_error(LB_EINVAL, "null network");
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status mlp_init(mlp_net** out, int seed, void* hip_stream) {
    if (!out) return lbk::set_error(LB_EINVAL, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return lbk::set_error(LB_EDEVICE, "no HIP device");
    mlp_net* n = new mlp_net();
    n->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        return lbk::set_error(LB_EDEVICE, "no current HIP device");
    }
    const long np = param_count();
    auto bail = [&](lb_status st) {
        mlp_free(n);
        return st;
    };
    if (hipMalloc(&n->P, sizeof(float) * np) != hipSuccess || hipMalloc(&n->G, sizeof(float) * np) != hipSuccess ||
        hipMalloc(&n->Mo, sizeof(float) * np) != hipSuccess || hipMalloc(&n->Vo, sizeof(float) * np) != hipSuccess)
        return bail(lbk::set_error(LB_ENOMEM, "device allocation of the network failed"));
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases
    std::vector<float> h(np);
    for (int l = 0; l < NLAYER; ++l) {
        const double bound = 1.0 / std::sqrt((double)DIMS[l]);
        const long a = w_off(l), b = b_off(l) + DIMS[l + 1];
        for (long i = a; i < b; ++i) h[i] = (float)((2.0 * uniform01((uint64_t)seed, (uint64_t)i) - 1.0) * bound);
    }
    if (hipMemcpy(n->P, h.data(), sizeof(float) * np, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->G, 0, sizeof(float) * np) != hipSuccess || hipMemset(n->Mo, 0, sizeof(float) * np) != hipSuccess ||
        hipMemset(n->Vo, 0, sizeof(float) * np) != hipSuccess)
        return bail(lbk::set_error(LB_EDEVICE, "network initialisation failed"));
    // set-up of the allocation-free inference path on this device
    float* sc = nullptr;
    if (lb_status st = noalloc_scratch(n->device, &sc)) return bail(st);
    *out = n;
    return LB_OK;
}

void mlp_free(mlp_net* n) {
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    else (void)hipDeviceSynchronize();
    free_rows(n);
    (void)hipFree(n->P);
    (void)hipFree(n->G);
    (void)hipFree(n->Mo);
    (void)hipFree(n->Vo);
    (void)hipFree(n->loss);
    (void)hipFree(n->Xall);
    (void)hipFree(n->Yall);
    (void)hipFree(n->idx);
    delete n;
}

long mlp_param_count(const mlp_net* n) { return n ? param_count() : 0; }

lb_status mlp_get_params(mlp_net* n, float* host, long count) {
    if (lb_status st = check_net(n)) return st;
    if (!host || count != param_count()) return lbk::set_error(LB_EINVAL, "parameter buffer size mismatch");
    MLP_TRY(hipMemcpyAsync(host, n->P, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
    MLP_TRY(hipStreamSynchronize(n->stream));
    return LB_OK;
}

lb_status mlp_set_params(mlp_net* n, const float* host, long count) {
    if (lb_status st = check_net(n)) return st;
    if (!host || count != param_count()) return lbk::set_error(LB_EINVAL, "parameter buffer size mismatch");
    MLP_TRY(hipMemcpyAsync(n->P, host, sizeof(float) * count, hipMemcpyHostToDevice, n->stream));
    MLP_TRY(hipMemsetAsync(n->Mo, 0, sizeof(float) * count, n->stream));
    MLP_TRY(hipMemsetAsync(n->Vo, 0, sizeof(float) * count, n->stream));
    MLP_TRY(hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    return LB_OK;
}

lb_status mlp_predict(mlp_net* n, const float* X, int rows, float* Y) {
    if (lb_status st = check_net(n)) return st;
    if (rows < 0 || (rows > 0 && (!X || !Y))) return lbk::set_error(LB_EINVAL, "bad rows or null arrays");
    if (rows == 0) return LB_OK;
    if (lb_status st = ensure_rows(n, rows)) return st;
    MLP_TRY(hipMemcpyAsync(n->act[0], X, sizeof(float) * (size_t)rows * DIMS[0], hipMemcpyHostToDevice, n->stream));
    if (lb_status st = forward(n, rows)) return st;
    MLP_TRY(hipMemcpyAsync(Y, n->z[NLAYER - 1], sizeof(float) * (size_t)rows * DIMS[NLAYER], hipMemcpyDeviceToHost,
                           n->stream));
    MLP_TRY(hipStreamSynchronize(n->stream));
    return LB_OK;
}

lb_status mlp_predict_device_noalloc(mlp_net* n, const float* dX, int rows, float* dY) {
    if (lb_status st = check_net(n)) return st;
    if (rows < 0 || rows > MLP_NOALLOC_MAX_ROWS)
        return lbk::set_error(LB_EINVAL, "mlp_predict_device_noalloc: rows must be in 0..MLP_NOALLOC_MAX_ROWS (1024)");
    if (rows > 0 && (!dX || !dY)) return lbk::set_error(LB_EINVAL, "null device arrays");
    if (rows == 0) return LB_OK;
    float* sc = nullptr;
    if (lb_status st = noalloc_scratch(n->device, &sc)) return st;
    // layer inputs: X, then the hidden activations alternating between the
    // second and third scratch buffers; pre-activations of the hidden layers
    // into the first (not read), the output straight into Y
    float* const a = sc + SCRATCH_BUF;
    float* const b = sc + 2 * SCRATCH_BUF;
    const float* const in[NLAYER] = {dX, a, b, a};
    float* const z[NLAYER] = {sc, sc, sc, dY};
    return forward_bufs(n->stream, n->P, rows, in, z);
}

lb_status mlp_loss_grad(mlp_net* n, const float* X, const float* Y, int rows, float* loss, float* grads) {
    if (lb_status st = check_net(n)) return st;
    if (rows <= 0 || !X || !Y) return lbk::set_error(LB_EINVAL, "bad rows or null arrays");
    if (lb_status st = ensure_rows(n, rows)) return st;
    if (lb_status st = ensure_loss(n, 1)) return st;
    MLP_TRY(hipMemcpyAsync(n->act[0], X, sizeof(float) * (size_t)rows * DIMS[0], hipMemcpyHostToDevice, n->stream));
    MLP_TRY(hipMemcpyAsync(n->yb, Y, sizeof(float) * (size_t)rows * DIMS[NLAYER], hipMemcpyHostToDevice, n->stream));
    if (lb_status st = forward(n, rows)) return st;
    if (lb_status st = mse(n, rows, n->loss)) return st;
    if (lb_status st = backward(n, rows)) return st;
    float l = 0.f;
    MLP_TRY(hipMemcpyAsync(&l, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    if (grads)
        MLP_TRY(hipMemcpyAsync(grads, n->G, sizeof(float) * param_count(), hipMemcpyDeviceToHost, n->stream));
    MLP_TRY(hipStreamSynchronize(n->stream));
    if (loss) *loss = l;
    return LB_OK;
}

lb_status mlp_train(mlp_net* n, const float* X, const float* Y, int rows, int epochs, int batch, float lr, int seed,
                    float* last_loss) {
    if (lb_status st = check_net(n)) return st;
    if (rows <= 0 || !X || !Y || epochs < 0 || batch <= 0 || !(lr > 0.f))
        return lbk::set_error(LB_EINVAL, "bad training arguments");
    const int nb = (rows + batch - 1) / batch;   // minibatches per epoch, the last one may be short
    const int bmax = std::min(batch, rows);
    if (lb_status st = ensure_rows(n, bmax)) return st;
    if (lb_status st = ensure_loss(n, nb)) return st;
    if (rows > n->data_cap) {
        MLP_TRY(hipStreamSynchronize(n->stream));
        (void)hipFree(n->Xall);
        (void)hipFree(n->Yall);
        (void)hipFree(n->idx);
        n->Xall = n->Yall = nullptr;
        n->idx = nullptr;
        n->data_cap = 0;
        MLP_TRY(hipMalloc(&n->Xall, sizeof(float) * (size_t)rows * DIMS[0]));
        MLP_TRY(hipMalloc(&n->Yall, sizeof(float) * (size_t)rows * DIMS[NLAYER]));
        MLP_TRY(hipMalloc(&n->idx, sizeof(int) * (size_t)rows));
        n->data_cap = rows;
    }
    MLP_TRY(hipMemcpyAsync(n->Xall, X, sizeof(float) * (size_t)rows * DIMS[0], hipMemcpyHostToDevice, n->stream));
    MLP_TRY(hipMemcpyAsync(n->Yall, Y, sizeof(float) * (size_t)rows * DIMS[NLAYER], hipMemcpyHostToDevice, n->stream));
    const long np = param_count();
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    std::vector<int> perm(rows);
    for (int e = 0; e < epochs; ++e) {
        // seeded Fisher-Yates shuffle of the rows
        for (int i = 0; i < rows; ++i) perm[i] = i;
        for (int i = rows - 1; i > 0; --i) {
            const uint64_t r = splitmix64(((uint64_t)seed << 32) ^ ((uint64_t)e * 0x9E3779B97F4A7C15ull) ^ (uint64_t)i);
            std::swap(perm[i], perm[(int)(r % (uint64_t)(i + 1))]);
        }
        MLP_TRY(hipStreamSynchronize(n->stream));   // the previous epoch's index upload has been consumed
        MLP_TRY(hipMemcpy(n->idx, perm.data(), sizeof(int) * (size_t)rows, hipMemcpyHostToDevice));
        for (int b = 0; b < nb; ++b) {
            const int r0 = b * batch, nr = std::min(batch, rows - r0);
            hipLaunchKernelGGL(mlp_gather, dim3(nr), dim3(64), 0, n->stream, n->Xall, n->Yall, n->idx + r0, nr,
                               DIMS[0], DIMS[NLAYER], n->act[0], n->yb);
            MLP_TRY(hipGetLastError());
            if (lb_status st = forward(n, nr)) return st;
            if (lb_status st = mse(n, nr, n->loss + b)) return st;
            if (lb_status st = backward(n, nr)) return st;
            n->adam_t += 1;
            const float bc1 = 1.f - (float)std::pow(0.9, (double)n->adam_t);
            const float bc2 = 1.f - (float)std::pow(0.999, (double)n->adam_t);
            hipLaunchKernelGGL(mlp_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, n->stream, n->P, n->G,
                               n->Mo, n->Vo, np, lr, b1, b2, eps, bc1, bc2);
            MLP_TRY(hipGetLastError());
        }
    }
    if (last_loss) {
        *last_loss = 0.f;
        if (epochs > 0) {
            std::vector<float> l(nb);
            MLP_TRY(hipMemcpyAsync(l.data(), n->loss, sizeof(float) * nb, hipMemcpyDeviceToHost, n->stream));
            MLP_TRY(hipStreamSynchronize(n->stream));
            double s = 0.0;
            for (int b = 0; b < nb; ++b) s += (double)l[b] * std::min(batch, rows - b * batch);
            *last_loss = (float)(s / rows);
        }
    }
    MLP_TRY(hipStreamSynchronize(n->stream));
    return LB_OK;
}

}  // extern "C"
