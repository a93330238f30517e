// Learned troubled-cell indicator: a small network n_inputs -> H -> H -> 1
// (tanh, tanh, sigmoid) over the modal-energy features of the smoothness
// indicator (Sec. 4), with hand-written inference and training kernels.
//
//   k_mlp_forward   one lane per row: the network's output
//   k_mlp_grad      one wavefront per workgroup, tiles of 64 rows: forward and
//                   reverse pass per row (one lane per row), activations and
//                   back-propagated errors staged in LDS, then each lane sums
//                   its parameters' products over the tile's rows (FP64
//                   accumulators), one partial row per workgroup
//   k_mlp_reduce    parameter-wise sum of the partial rows (fixed order), scaled
//   k_mlp_adam      Adam update of the parameters from the reduced gradient
//   k_mlp_box       per-feature min / max of a data set (the feature box)
//
// Loss: mean squared error over the rows.  Parameters per layer: W[out][in]
// row-major, then b[out].  Everything runs on the network's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/crkfr.h"
#include "crkfr_internal.hpp"
#include "crkfr_kernels.hpp"

using namespace crkfr;

struct crkfr_mlp {
    int nin, H, npar;
    hipStream_t stream;
    bool own_stream;
    float* params;       // npar network parameters, then lo[nin], hi[nin]
    float* adam_m;
    float* adam_v;
    double* part;        // partial sums [part_rows][npar + 1] (last column: sum of squared residuals)
    int part_rows;
    float* grad;         // reduced gradient [npar], then the mean loss
    double* loss_acc;    // per-epoch loss accumulators
    int loss_cap;
    long long adam_t;
};

namespace crkfr {
const float* mlp_device_params(const crkfr_mlp* m) { return m->params; }
int mlp_inputs(const crkfr_mlp* m) { return m->nin; }
int mlp_hidden(const crkfr_mlp* m) { return m->H; }
}  // namespace crkfr

#define MLP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(CRKFR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

namespace {

constexpr int TILE = 64;          // rows per tile = lanes per workgroup in k_mlp_grad
constexpr int LROW = TILE + 1;    // padded LDS row (rows of one tile land in different banks)
constexpr int GRAD_WG_MAX = 512;  // partial rows (workgroups) of one gradient pass

template <int NIN, int H>
__device__ __forceinline__ float mlp_eval(const float* __restrict__ P, const float* x, float* h1, float* h2)
{
    const float* W1 = P;
    const float* b1 = W1 + H * NIN;
    const float* W2 = b1 + H;
    const float* b2 = W2 + H * H;
    const float* w3 = b2 + H;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = b1[j];
#pragma unroll
        for (int i = 0; i < NIN; ++i) s += W1[j * NIN + i] * x[i];
        h1[j] = tanhf(s);
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = b2[j];
#pragma unroll
        for (int i = 0; i < H; ++i) s += W2[j * H + i] * h1[i];
        h2[j] = tanhf(s);
    }
    float s = w3[H];
#pragma unroll
    for (int j = 0; j < H; ++j) s += w3[j] * h2[j];
    return 1.0f / (1.0f + expf(-s));
}

template <int NIN, int H>
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ P, const float* __restrict__ x, int n,
                                                     float* __restrict__ y)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float xi[NIN], h1[H], h2[H];
#pragma unroll
    for (int i = 0; i < NIN; ++i) xi[i] = x[(size_t)r * NIN + i];
    y[r] = mlp_eval<NIN, H>(P, xi, h1, h2);
}

// gradient of the summed squared residual over rows [base, base + count)
template <int NIN, int H>
__global__ void __launch_bounds__(TILE) k_mlp_grad(const float* __restrict__ P, const float* __restrict__ x,
                                                   const float* __restrict__ t, int base, int count,
                                                   double* __restrict__ part)
{
    constexpr int NPAR = mlp_nparams(NIN, H);
    constexpr int NACC = NPAR + 1;                       // + squared residual
    constexpr int PPL = (NACC + TILE - 1) / TILE;        // accumulators per lane
    // LDS rows: x (NIN), h1 (H), d1 (H), h2 (H), d2 (H), d3, r^2, ones
    constexpr int R_X = 0, R_H1 = NIN, R_D1 = R_H1 + H, R_H2 = R_D1 + H, R_D2 = R_H2 + H, R_D3 = R_D2 + H;
    constexpr int R_L = R_D3 + 1, R_ONE = R_L + 1, NROW = R_ONE + 1;
    __shared__ float lds[NROW * LROW];
    const int lane = threadIdx.x;
    const float* W2 = P + H * NIN + H;
    const float* w3 = W2 + H * H + H;

    // each accumulator slot is a sum over rows of lds[a][row] * lds[b][row]
    int ra[PPL], rb[PPL];
#pragma unroll
    for (int s = 0; s < PPL; ++s) {
        int p = lane + s * TILE, a = R_ONE, b = R_ONE;
        if (p < H * NIN) { a = R_D1 + p / NIN; b = R_X + p % NIN; }
        else if ((p -= H * NIN) < H) { a = R_D1 + p; }
        else if ((p -= H) < H * H) { a = R_D2 + p / H; b = R_H1 + p % H; }
        else if ((p -= H * H) < H) { a = R_D2 + p; }
        else if ((p -= H) < H) { a = R_D3; b = R_H2 + p; }
        else if ((p -= H) == 0) { a = R_D3; }
        else if (p == 1) { a = R_L; }
        ra[s] = a;
        rb[s] = b;
    }
    double acc[PPL];
#pragma unroll
    for (int s = 0; s < PPL; ++s) acc[s] = 0.0;
    lds[R_ONE * LROW + lane] = 1.0f;

    const int ntiles = (count + TILE - 1) / TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int row = tile * TILE + lane;
        const bool valid = row < count;
        float xi[NIN], h1[H], h2[H], d1[H], d2[H];
#pragma unroll
        for (int i = 0; i < NIN; ++i) xi[i] = valid ? x[(size_t)(base + row) * NIN + i] : 0.0f;
        const float y = mlp_eval<NIN, H>(P, xi, h1, h2);
        const float r = valid ? y - t[base + row] : 0.0f;
        const float d3 = 2.0f * r * y * (1.0f - y);
#pragma unroll
        for (int j = 0; j < H; ++j) d2[j] = d3 * w3[j] * (1.0f - h2[j] * h2[j]);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < H; ++j) s += W2[j * H + i] * d2[j];
            d1[i] = s * (1.0f - h1[i] * h1[i]);
        }
#pragma unroll
        for (int i = 0; i < NIN; ++i) lds[(R_X + i) * LROW + lane] = xi[i];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            lds[(R_H1 + j) * LROW + lane] = h1[j];
            lds[(R_D1 + j) * LROW + lane] = d1[j];
            lds[(R_H2 + j) * LROW + lane] = h2[j];
            lds[(R_D2 + j) * LROW + lane] = d2[j];
        }
        lds[R_D3 * LROW + lane] = d3;
        lds[R_L * LROW + lane] = r * r;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PPL; ++s) {
            const float* A = &lds[ra[s] * LROW];
            const float* B = &lds[rb[s] * LROW];
            float sum = 0.0f;
            for (int q = 0; q < TILE; ++q) sum += A[q] * B[q];
            acc[s] += (double)sum;
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < PPL; ++s) {
        int p = lane + s * TILE;
        if (p < NACC) part[(size_t)blockIdx.x * NACC + p] = acc[s];
    }
}

// grad[p] = scale * sum over partial rows (fixed order)
__global__ void __launch_bounds__(256) k_mlp_reduce(const double* __restrict__ part, int rows, int nacc, double scale,
                                                    float* __restrict__ grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nacc) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += part[(size_t)r * nacc + p];
    grad[p] = (float)(s * scale);
}

struct AdamArgs {
    float lr, beta1, beta2, eps, bc1, bc2;
    int npar;
    double* loss_acc;
    double loss_weight;
};

__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ grad, AdamArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *a.loss_acc += a.loss_weight * (double)grad[a.npar];
    if (p >= a.npar) return;
    const float g = grad[p];
    const float mm = a.beta1 * m[p] + (1.0f - a.beta1) * g;
    const float vv = a.beta2 * v[p] + (1.0f - a.beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    P[p] -= a.lr * (mm / a.bc1) / (sqrtf(vv / a.bc2) + a.eps);
}

// feature box: box[f] = min - margin, box[nin + f] = max + margin over rows
__global__ void __launch_bounds__(256) k_mlp_box(const float* __restrict__ x, int n, int nin, float margin,
                                                 float* __restrict__ box)
{
    __shared__ float smin[256], smax[256];
    const int f = blockIdx.x;
    float lo = INFINITY, hi = -INFINITY;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        float v = x[(size_t)r * nin + f];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + w]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        box[f] = smin[0] - margin;
        box[nin + f] = smax[0] + margin;
    }
}

// ---- dispatch over (inputs, hidden) ----
enum { K_FORWARD, K_GRAD };

struct Launch {
    int kind;
    const float* P;
    const float* x;
    const float* t;
    float* y;
    int n, base, count, grid;
    double* part;
};

template <int NIN, int H>
void launch_t(const Launch& L, hipStream_t st)
{
    if (L.kind == K_FORWARD)
        hipLaunchKernelGGL((k_mlp_forward<NIN, H>), dim3((L.n + 255) / 256), dim3(256), 0, st, L.P, L.x, L.n, L.y);
    else
        hipLaunchKernelGGL((k_mlp_grad<NIN, H>), dim3(L.grid), dim3(TILE), 0, st, L.P, L.x, L.t, L.base, L.count,
                           L.part);
}

template <int NIN>
int launch_h(int H, const Launch& L, hipStream_t st)
{
    switch (H) {
    case 8: launch_t<NIN, 8>(L, st); return 0;
    case 16: launch_t<NIN, 16>(L, st); return 0;
    case 32: launch_t<NIN, 32>(L, st); return 0;
    }
    return -1;
}

int launch(const crkfr_mlp* m, const Launch& L)
{
    int rc = -1;
    switch (m->nin) {
    case 1: rc = launch_h<1>(m->H, L, m->stream); break;
    case 2: rc = launch_h<2>(m->H, L, m->stream); break;
    case 3: rc = launch_h<3>(m->H, L, m->stream); break;
    case 4: rc = launch_h<4>(m->H, L, m->stream); break;
    }
    if (rc) return set_error(CRKFR_EINVAL, "no network kernel for this size");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CRKFR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return 0;
}

// splitmix64 (Steele, Lea, Flood 2014) for the initial weights
uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void free_mlp(crkfr_mlp* m)
{
    void* ptrs[] = {m->params, m->adam_m, m->adam_v, m->part, m->grad, m->loss_acc};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
}

// gradient of the mean squared error over rows [base, base + count) into m->grad
int grad_pass(crkfr_mlp* m, const float* x, const float* t, int base, int count)
{
    Launch L{};
    L.kind = K_GRAD;
    L.P = m->params;
    L.x = x;
    L.t = t;
    L.base = base;
    L.count = count;
    const int tiles = (count + TILE - 1) / TILE;
    L.grid = tiles < GRAD_WG_MAX ? tiles : GRAD_WG_MAX;
    L.part = m->part;
    int rc = launch(m, L);
    if (rc) return rc;
    const int nacc = m->npar + 1;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((nacc + 255) / 256), dim3(256), 0, m->stream, m->part, L.grid, nacc,
                       1.0 / count, m->grad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CRKFR_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return 0;
}

}  // namespace

extern "C" int crkfr_mlp_create(int n_inputs, int hidden, unsigned long long seed, void* hip_stream,
                                crkfr_mlp** out)
{
    if (!out) return set_error(CRKFR_EINVAL, "null argument");
    *out = nullptr;
    if (n_inputs < 1 || n_inputs > 4) return set_error(CRKFR_EINVAL, "n_inputs must be in 1..4 (the degree N)");
    if (hidden != 8 && hidden != 16 && hidden != 32) return set_error(CRKFR_EINVAL, "hidden must be 8, 16 or 32");
    crkfr_mlp* m = new crkfr_mlp();
    std::memset(m, 0, sizeof(*m));
    m->nin = n_inputs;
    m->H = hidden;
    m->npar = mlp_nparams(n_inputs, hidden);
    m->stream = (hipStream_t)hip_stream;
    if (!m->stream) {
        hipError_t e = hipStreamCreate(&m->stream);
        if (e != hipSuccess) {
            delete m;
            return set_error(CRKFR_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        m->own_stream = true;
    }
    m->part_rows = GRAD_WG_MAX;
    bool ok = hipMalloc((void**)&m->params, (m->npar + 2 * m->nin) * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->adam_m, m->npar * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->adam_v, m->npar * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->part, (size_t)m->part_rows * (m->npar + 1) * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void**)&m->grad, (m->npar + 1) * sizeof(float)) == hipSuccess;
    if (!ok) {
        free_mlp(m);
        delete m;
        return set_error(CRKFR_ENOMEM, "device allocation failed");
    }
    // Glorot-uniform weights, zero biases; the feature box is the features' full range [-1, 1]
    std::vector<float> h(m->npar + 2 * m->nin, 0.0f);
    uint64_t st = seed;
    const int dims[4] = {m->nin, m->H, m->H, 1};
    int off = 0;
    for (int l = 0; l < 3; ++l) {
        const double lim = std::sqrt(6.0 / (dims[l] + dims[l + 1]));
        for (int i = 0; i < dims[l] * dims[l + 1]; ++i) {
            double u = (splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            h[off + i] = (float)((2.0 * u - 1.0) * lim);
        }
        off += dims[l] * dims[l + 1] + dims[l + 1];
    }
    for (int f = 0; f < m->nin; ++f) {
        h[m->npar + f] = -1.0f;
        h[m->npar + m->nin + f] = 1.0f;
    }
    hipError_t e = hipMemcpyAsync(m->params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->adam_m, 0, m->npar * sizeof(float), m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->adam_v, 0, m->npar * sizeof(float), m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        free_mlp(m);
        delete m;
        return set_error(CRKFR_EHIP, std::string("network set-up: ") + hipGetErrorString(e));
    }
    *out = m;
    return 0;
}

extern "C" void crkfr_mlp_destroy(crkfr_mlp* m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    free_mlp(m);
    delete m;
}

extern "C" int crkfr_mlp_num_params(const crkfr_mlp* m) { return m ? m->npar : 0; }

extern "C" int crkfr_mlp_set_params(crkfr_mlp* m, const float* params, int on_device)
{
    if (!m || !params) return set_error(CRKFR_EINVAL, "null argument");
    MLP_TRY(hipMemcpyAsync(m->params, params, m->npar * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, m->stream));
    MLP_TRY(hipMemsetAsync(m->adam_m, 0, m->npar * sizeof(float), m->stream));
    MLP_TRY(hipMemsetAsync(m->adam_v, 0, m->npar * sizeof(float), m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    m->adam_t = 0;
    return 0;
}

extern "C" int crkfr_mlp_get_params(crkfr_mlp* m, float* params, int on_device)
{
    if (!m || !params) return set_error(CRKFR_EINVAL, "null argument");
    MLP_TRY(hipMemcpyAsync(params, m->params, m->npar * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    return 0;
}

extern "C" int crkfr_mlp_set_box(crkfr_mlp* m, const float* lo, const float* hi)
{
    if (!m || !lo || !hi) return set_error(CRKFR_EINVAL, "null argument");
    std::vector<float> b(2 * m->nin);
    for (int f = 0; f < m->nin; ++f) {
        b[f] = lo[f];
        b[m->nin + f] = hi[f];
    }
    MLP_TRY(hipMemcpyAsync(m->params + m->npar, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    return 0;
}

extern "C" int crkfr_mlp_get_box(crkfr_mlp* m, float* lo, float* hi)
{
    if (!m || !lo || !hi) return set_error(CRKFR_EINVAL, "null argument");
    std::vector<float> b(2 * m->nin);
    MLP_TRY(hipMemcpyAsync(b.data(), m->params + m->npar, b.size() * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    for (int f = 0; f < m->nin; ++f) {
        lo[f] = b[f];
        hi[f] = b[m->nin + f];
    }
    return 0;
}

extern "C" int crkfr_mlp_fit_box(crkfr_mlp* m, const float* x, int n, float margin)
{
    if (!m || !x) return set_error(CRKFR_EINVAL, "null argument");
    if (n < 1 || !(margin >= 0.0f)) return set_error(CRKFR_EINVAL, "need n >= 1 rows and margin >= 0");
    hipLaunchKernelGGL(k_mlp_box, dim3(m->nin), dim3(256), 0, m->stream, x, n, m->nin, margin, m->params + m->npar);
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipStreamSynchronize(m->stream));
    return 0;
}

extern "C" int crkfr_mlp_forward(crkfr_mlp* m, const float* x, int n, float* y)
{
    if (!m || !x || !y) return set_error(CRKFR_EINVAL, "null argument");
    if (n < 0) return set_error(CRKFR_EINVAL, "n < 0");
    if (n == 0) return 0;
    Launch L{};
    L.kind = K_FORWARD;
    L.P = m->params;
    L.x = x;
    L.y = y;
    L.n = n;
    return launch(m, L);
}

extern "C" int crkfr_mlp_loss_grad(crkfr_mlp* m, const float* x, const float* t, int n, double* loss, float* grad)
{
    if (!m || !x || !t) return set_error(CRKFR_EINVAL, "null argument");
    if (n < 1) return set_error(CRKFR_EINVAL, "need n >= 1 rows");
    int rc = grad_pass(m, x, t, 0, n);
    if (rc) return rc;
    std::vector<float> g(m->npar + 1);
    MLP_TRY(hipMemcpyAsync(g.data(), m->grad, g.size() * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    if (grad) std::memcpy(grad, g.data(), m->npar * sizeof(float));
    if (loss) *loss = g[m->npar];
    return 0;
}

extern "C" int crkfr_mlp_train(crkfr_mlp* m, const float* x, const float* t, int n, int epochs, int batch, float lr,
                               float* loss_per_epoch)
{
    if (!m || !x || !t) return set_error(CRKFR_EINVAL, "null argument");
    if (n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0f))
        return set_error(CRKFR_EINVAL, "need n, epochs, batch >= 1 and lr > 0");
    if (m->loss_cap < epochs) {
        if (m->loss_acc) (void)hipFree(m->loss_acc);
        m->loss_acc = nullptr;
        m->loss_cap = 0;
        MLP_TRY(hipMalloc((void**)&m->loss_acc, epochs * sizeof(double)));
        m->loss_cap = epochs;
    }
    MLP_TRY(hipMemsetAsync(m->loss_acc, 0, epochs * sizeof(double), m->stream));
    const float b1 = 0.9f, b2 = 0.999f;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int base = 0; base < n; base += batch) {
            const int cnt = n - base < batch ? n - base : batch;
            int rc = grad_pass(m, x, t, base, cnt);
            if (rc) return rc;
            ++m->adam_t;
            AdamArgs a;
            a.lr = lr;
            a.beta1 = b1;
            a.beta2 = b2;
            a.eps = 1e-8f;
            a.bc1 = (float)(1.0 - std::pow((double)b1, (double)m->adam_t));
            a.bc2 = (float)(1.0 - std::pow((double)b2, (double)m->adam_t));
            a.npar = m->npar;
            a.loss_acc = m->loss_acc + ep;
            a.loss_weight = (double)cnt / n;
            hipLaunchKernelGGL(k_mlp_adam, dim3((m->npar + 255) / 256), dim3(256), 0, m->stream, m->params,
                               m->adam_m, m->adam_v, m->grad, a);
            MLP_TRY(hipGetLastError());
        }
    }
    std::vector<double> l(epochs);
    MLP_TRY(hipMemcpyAsync(l.data(), m->loss_acc, epochs * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    MLP_TRY(hipStreamSynchronize(m->stream));
    if (loss_per_epoch)
        for (int i = 0; i < epochs; ++i) loss_per_epoch[i] = (float)l[i];
    return 0;
}
