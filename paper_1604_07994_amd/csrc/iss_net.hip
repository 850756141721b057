// Learned interface-band correction: a 3-layer 3x3x3 convolution network
// (8 -> 16 -> 16 -> 4 channels, ReLU, no biases) evaluated on the band of
// lattice vertices within Chebyshev distance 2 of the viscosity interface,
// trained on (residual, error) pairs produced by the solver.
//
// Layout: activations live on the dense lattice, channel-last, in BF16
// (act[v * C + c]); vertices off the band hold zeros, which gives the zero
// padding of the convolution.  A layer is an implicit GEMM with
//   M = band vertices, K = 27 taps x C_in (k = tap * C_in + c), N = C_out,
// computed with v_mfma_f32_16x16x16bf16_1k (BF16 operands, FP32
// accumulation): one wavefront owns 16 band vertices x 16 output channels and
// walks K in chunks of 16.  Weight fragments are pre-swizzled once per
// weight update.  Backward: dW is the GEMM dZ^T x im2col(A) reduced over the
// band in two deterministic stages; dA is the same convolution with
// transposed, tap-flipped weights, masked by the ReLU of the layer below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/iss.h"
#include "iss_internal.h"

namespace iss {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

constexpr int NET_CIN = 8, NET_CH = 16, NET_COUT = 4;

struct NetGeom {
    int n;                 // cells per axis; lattice (n+1)^3
    int64_t N, sy, sz;
    int64_t M;             // band vertices
    const int32_t* band;   // band vertex ids
    double h, beta;        // mesh width, stabilisation constant
};

__device__ __forceinline__ int64_t tap_vertex(const NetGeom& g, int64_t v, int tap, bool& ok) {
    const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
    const int64_t n1 = g.n + 1;
    const int i = (int)(v % n1), j = (int)((v / n1) % n1), k = (int)(v / (n1 * n1));
    ok = (i + dx >= 0) && (i + dx <= g.n) && (j + dy >= 0) && (j + dy <= g.n) && (k + dz >= 0) && (k + dz <= g.n);
    return v + dx + dy * g.sy + dz * g.sz;
}

// ---------------------------------------------------------------------------
// convolution layer (forward, or backward-data with flipped weights)
//   in:  dense BF16, CI channels per vertex (CI multiple of 4)
//   wB:  swizzled BF16 B fragments, [KC][64 lanes][4]
//   OUT_MODE 0: act_out[band[m]*CO + co] = bf16(relu(z))
//   OUT_MODE 1: yf[m*CO + co] = z (fp32, band order)
//   OUT_MODE 2: act_out[band[m]*CO + co] = bf16(z * (mask[band[m]*CO + co] > 0))
template <int CI, int CO, int OUT_MODE>
__global__ __launch_bounds__(256) void k_conv(NetGeom g, const uint16_t* __restrict__ in,
                                              const uint16_t* __restrict__ wB,
                                              uint16_t* __restrict__ act_out, float* __restrict__ yf,
                                              const uint16_t* __restrict__ mask) {
    constexpr int KC = (27 * CI + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (m0 >= g.M) return;
    const int r = lane & 15, q = lane >> 4;
    const int64_t ma = m0 + r;
    const int64_t va = (ma < g.M) ? g.band[ma] : -1;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const bf16x4* wf = reinterpret_cast<const bf16x4*>(wB);
    for (int kc = 0; kc < KC; ++kc) {
        const int k0 = kc * 16 + 4 * q;
        const int tap = k0 / CI, c0 = k0 % CI;
        bf16x4 a = {0, 0, 0, 0};
        if (va >= 0 && tap < 27) {
            bool ok;
            const int64_t u = tap_vertex(g, va, tap, ok);
            if (ok) a = *reinterpret_cast<const bf16x4*>(in + u * CI + c0);
        }
        const bf16x4 b = wf[kc * 64 + lane];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int co = lane & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + 4 * q + i;
        if (m >= g.M || co >= CO) continue;
        const float z = acc[i];
        if (OUT_MODE == 1) {
            yf[m * CO + co] = z;
        } else {
            const int64_t v = g.band[m];
            float o = z;
            if (OUT_MODE == 0) o = fmaxf(z, 0.f);
            if (OUT_MODE == 2) o = (bf2f(mask[v * CO + co]) > 0.f) ? z : 0.f;
            act_out[v * CO + co] = f2bf(o);
        }
    }
}

// Swizzle FP32 weights W[co][ci][tap] into B fragments: lane l of chunk kc
// holds B[k = kc*16 + 4*(l/16) + i][n = l%16].  flip = 1 gives the weights of
// the backward-data convolution: B'[k = tap*CO + co][n = ci] = W[co][ci][26-tap].
template <int CI, int CO>
__global__ void k_swizzle(const float* __restrict__ W, uint16_t* __restrict__ wB, int flip) {
    // forward: input channels CI, outputs CO; flipped: input CO, outputs CI
    const int cin = flip ? CO : CI, cout = flip ? CI : CO;
    const int KC = (27 * cin + 15) / 16;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= KC * 64 * 4) return;
    const int i = e & 3, l = (e >> 2) & 63, kc = e >> 8;
    const int k = kc * 16 + 4 * (l >> 4) + i, nn = l & 15;
    float w = 0.f;
    const int tap = k / cin, c = k % cin;
    if (tap < 27 && nn < cout) {
        if (!flip) w = W[((int64_t)nn * CI + c) * 27 + tap];
        else w = W[((int64_t)c * CI + nn) * 27 + (26 - tap)];
    }
    wB[e] = f2bf(w);
}

// dW[co][ci][tap] partial sums over a block of 64 band vertices:
//   sum_m dz[m][co] * in[nb(m, tap)][ci]
// GEMM with M' = CO (rows), N' = 27*CI (cols), reduction over band vertices.
// One wavefront: 16 columns, 16 band vertices per MFMA step.
template <int CI, int CO>
__global__ __launch_bounds__(256) void k_wgrad(NetGeom g, const uint16_t* __restrict__ dz_dense,
                                               const uint16_t* __restrict__ in, float* __restrict__ partial,
                                               int64_t m_per_block) {
    constexpr int NCOLT = (27 * CI + 15) / 16;     // column tiles
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ct = blockIdx.y * 4 + wave;           // column tile of this wave
    const int64_t mb = (int64_t)blockIdx.x * m_per_block;
    const int64_t me = std::min<int64_t>(g.M, mb + m_per_block);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int q = lane >> 4, rr = lane & 15;
    const int col = ct * 16 + rr;                   // k' = tap*CI + ci for B
    const int tap = col / CI, ci = col % CI;
    if (ct < NCOLT) {
        for (int64_t m0 = mb; m0 < me; m0 += 16) {
            bf16x4 a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t m = m0 + 4 * q + i;
                uint16_t av = 0, bv = 0;
                if (m < me) {
                    const int64_t v = g.band[m];
                    if (rr < CO) av = dz_dense[v * CO + rr];          // A[row = co][m]
                    if (tap < 27) {
                        bool ok;
                        const int64_t u = tap_vertex(g, v, tap, ok);
                        if (ok) bv = in[u * CI + ci];                 // B[m][col]
                    }
                }
                a[i] = (short)av;
                b[i] = (short)bv;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
    }
    // D[row = 4q + i][col = rr]: row = co, col within tile
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int co = 4 * q + i;
        if (ct < NCOLT && co < CO && col < 27 * CI) {
            const int t2 = col / CI, c2 = col % CI;
            partial[(int64_t)blockIdx.x * (CO * CI * 27) + ((int64_t)co * CI + c2) * 27 + t2] = acc[i];
        }
    }
}

__global__ void k_sum_blocks(const float* __restrict__ partial, int nblk, int64_t len,
                             float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * len + e];
    out[e] = (float)s;
}

// features of the band vertices from a residual r (FP64, (d+1) N):
// channels r_u/s_u, r_v/s_u, r_w/s_u, r_p/s_p, log10(mu)/4, interface, 0, 0
__global__ void k_band_sumsq(NetGeom g, const double* __restrict__ r, double* __restrict__ partial) {
    __shared__ double sh[2][4];
    double su = 0, sp = 0;
    for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < g.M; m += (int64_t)gridDim.x * 256) {
        const int64_t v = g.band[m];
        for (int c = 0; c < 3; ++c) { const double t = r[c * g.N + v]; su += t * t; }
        const double t = r[3 * g.N + v];
        sp += t * t;
    }
    for (int o = 32; o > 0; o >>= 1) { su += __shfl_down(su, o, 64); sp += __shfl_down(sp, o, 64); }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sh[0][w] = su; sh[1][w] = sp; }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 2 + 0] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        partial[blockIdx.x * 2 + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

__global__ void k_band_scales(const double* __restrict__ partial, int nblk, int64_t M, double* __restrict__ scales) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double su = 0, sp = 0;
    for (int b = 0; b < nblk; ++b) { su += partial[2 * b]; sp += partial[2 * b + 1]; }
    const double mm = (double)(M > 0 ? M : 1);
    su = sqrt(su / (3.0 * mm));
    sp = sqrt(sp / mm);
    scales[0] = su > 0 ? su : 1.0;
    scales[1] = sp > 0 ? sp : 1.0;
}

__global__ void k_band_features(NetGeom g, const double* __restrict__ r, const double* __restrict__ scales,
                                const float* __restrict__ static_feat, uint16_t* __restrict__ act0) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    const int64_t v = g.band[m];
    const double iu = 1.0 / scales[0], ip = 1.0 / scales[1];
    uint16_t* o = act0 + v * NET_CIN;
    o[0] = f2bf((float)(r[v] * iu));
    o[1] = f2bf((float)(r[g.N + v] * iu));
    o[2] = f2bf((float)(r[2 * g.N + v] * iu));
    o[3] = f2bf((float)(r[3 * g.N + v] * ip));
    o[4] = f2bf(static_feat[2 * m]);
    o[5] = f2bf(static_feat[2 * m + 1]);
    o[6] = 0;
    o[7] = 0;
}

// Jacobi units: the diagonal of an isoviscous row at the vertex's largest
// incident viscosity mu: 6 mu h (velocity component), 6 beta h^3 / mu (pressure)
__device__ __forceinline__ void diag_scales(const NetGeom& g, const float* static_feat, int64_t m,
                                            double& du, double& dp) {
    const double mu = pow(10.0, 4.0 * (double)static_feat[2 * m]);
    du = 6.0 * mu * g.h;
    dp = 6.0 * g.beta * g.h * g.h * g.h / mu;
}

__global__ void k_band_targets(NetGeom g, const double* __restrict__ e, const double* __restrict__ scales,
                               const float* __restrict__ static_feat, float* __restrict__ t) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    const int64_t v = g.band[m];
    double du, dp;
    diag_scales(g, static_feat, m, du, dp);
    for (int c = 0; c < 3; ++c) t[m * 4 + c] = (float)(e[c * g.N + v] * du / scales[0]);
    t[m * 4 + 3] = (float)(e[3 * g.N + v] * dp / scales[1]);
}

// dL/dy for the MSE loss and its value: dy = 2 (y - t) / (4 M)
__global__ void k_mse(NetGeom g, const float* __restrict__ y, const float* __restrict__ t,
                      uint16_t* __restrict__ dy_dense, double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc = 0;
    const double inv = 1.0 / (4.0 * (double)g.M);
    for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < g.M; m += (int64_t)gridDim.x * 256) {
        const int64_t v = g.band[m];
        for (int c = 0; c < 4; ++c) {
            const double d = (double)y[m * 4 + c] - (double)t[m * 4 + c];
            acc += d * d;
            dy_dense[v * 4 + c] = f2bf((float)(2.0 * d * inv));
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1] + sh[2] + sh[3]) * inv;
}

__global__ void k_sum_partial(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0;
        for (int b = 0; b < nblk; ++b) s += partial[b];
        out[0] = s;
    }
}

// z += correction: velocity (not on the boundary) and pressure
__global__ void k_band_correct(NetGeom g, const float* __restrict__ y, const double* __restrict__ scales,
                               const float* __restrict__ static_feat, double* __restrict__ z) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    const int64_t v = g.band[m];
    const int64_t n1 = g.n + 1;
    const int i = (int)(v % n1), j = (int)((v / n1) % n1), k = (int)(v / (n1 * n1));
    const bool bnd = i == 0 || j == 0 || k == 0 || i == g.n || j == g.n || k == g.n;
    double du, dp;
    diag_scales(g, static_feat, m, du, dp);
    if (!bnd)
        for (int c = 0; c < 3; ++c) z[c * g.N + v] += (double)y[m * 4 + c] * scales[0] / du;
    z[3 * g.N + v] += (double)y[m * 4 + 3] * scales[1] / dp;
}

// dL/dy from dL/dc for c = correction(y): dy[m][ch] = dLdc[ch][v] * s_ch / d_ch
// (velocity channels are 0 on the boundary, where c is not applied); the
// result goes to the dense BF16 array the backward pass reads.
__global__ void k_band_output_grad(NetGeom g, const double* __restrict__ dldc, double factor,
                                   const double* __restrict__ scales, const float* __restrict__ static_feat,
                                   uint16_t* __restrict__ dy_dense) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.M) return;
    const int64_t v = g.band[m];
    const int64_t n1 = g.n + 1;
    const int i = (int)(v % n1), j = (int)((v / n1) % n1), k = (int)(v / (n1 * n1));
    const bool bnd = i == 0 || j == 0 || k == 0 || i == g.n || j == g.n || k == g.n;
    double du, dp;
    diag_scales(g, static_feat, m, du, dp);
    for (int c = 0; c < 3; ++c)
        dy_dense[v * 4 + c] = f2bf(bnd ? 0.f : (float)(factor * dldc[c * g.N + v] * scales[0] / du));
    dy_dense[v * 4 + 3] = f2bf((float)(factor * dldc[3 * g.N + v] * scales[1] / dp));
}

__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ gr, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = gr[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

template <typename T>
__global__ void k_zero(T* __restrict__ x, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) x[e] = 0;
}

// band rows of the input activation (N x 8, BF16 bits) <-> compact M x 8
template <bool SAVE>
__global__ void k_band_rows(const int32_t* __restrict__ band, int64_t M, uint16_t* __restrict__ act0,
                            uint16_t* __restrict__ compact) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * NET_CIN) return;
    const int64_t m = e / NET_CIN;
    const int c = (int)(e - m * NET_CIN);
    const int64_t a = (int64_t)band[m] * NET_CIN + c;
    if (SAVE) compact[e] = act0[a];
    else act0[a] = compact[e];
}

}  // namespace iss

// ===========================================================================
// host side

namespace iss {

struct NetImpl {
    NetGeom g{};
    int64_t nparams = 0;
    int32_t* band = nullptr;
    float* static_feat = nullptr;
    uint16_t* act0 = nullptr;   // N x 8
    uint16_t* act1 = nullptr;   // N x 16
    uint16_t* act2 = nullptr;   // N x 16
    uint16_t* dz1 = nullptr;    // N x 16
    uint16_t* dz2 = nullptr;    // N x 16
    uint16_t* dy = nullptr;     // N x 4
    float* y = nullptr;         // M x 4
    uint16_t* wB[3] = {nullptr, nullptr, nullptr};
    uint16_t* wF[3] = {nullptr, nullptr, nullptr};   // flipped (layers 2, 3)
    float* partial = nullptr;
    double* dpartial = nullptr;
    double* scales = nullptr;   // device: s_u, s_p
    double* dloss = nullptr;
    double* h_pinned = nullptr;
    bool weights_set = false;
    // correction workspace (FP64 vectors of the finest level)
    double* rp = nullptr;
    double* cvec = nullptr;
    double* rpp = nullptr;
    std::vector<void*> allocs;
    int64_t wblocks = 0, m_per_block = 0;
};

static int kc_of(int cin) { return (27 * cin + 15) / 16; }

static hipError_t nalloc(NetImpl* n, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
    if (e == hipSuccess) n->allocs.push_back(*p);
    return e;
}

hipError_t net_create(const NetSetup& s, NetImpl** out) {
    NetImpl* n = new NetImpl();
    n->g.n = s.n;
    n->g.N = s.N;
    n->g.sy = s.n + 1;
    n->g.sz = (int64_t)(s.n + 1) * (s.n + 1);
    n->g.M = (int64_t)s.band.size();
    n->g.h = 1.0 / s.n;
    n->g.beta = s.beta;
    n->nparams = 16 * 8 * 27 + 16 * 16 * 27 + 4 * 16 * 27;
    hipError_t e;
#define NA(ptr, bytes) if ((e = nalloc(n, (void**)&(ptr), (bytes))) != hipSuccess) { net_destroy(n); return e; }
    NA(n->band, n->g.M * 4);
    NA(n->static_feat, n->g.M * 8);
    NA(n->act0, s.N * NET_CIN * 2);
    NA(n->act1, s.N * NET_CH * 2);
    NA(n->act2, s.N * NET_CH * 2);
    NA(n->dz1, s.N * NET_CH * 2);
    NA(n->dz2, s.N * NET_CH * 2);
    NA(n->dy, s.N * NET_COUT * 2);
    NA(n->y, n->g.M * NET_COUT * 4);
    NA(n->wB[0], kc_of(NET_CIN) * 64 * 4 * 2);
    NA(n->wB[1], kc_of(NET_CH) * 64 * 4 * 2);
    NA(n->wB[2], kc_of(NET_CH) * 64 * 4 * 2);
    NA(n->wF[1], kc_of(NET_CH) * 64 * 4 * 2);
    NA(n->wF[2], kc_of(NET_COUT) * 64 * 4 * 2);
    n->m_per_block = 1024;
    n->wblocks = std::max<int64_t>(1, (n->g.M + n->m_per_block - 1) / n->m_per_block);
    NA(n->partial, n->wblocks * 16 * 16 * 27 * 4);
    NA(n->dpartial, 2048 * 8);
    NA(n->scales, 2 * 8);
    NA(n->dloss, 8);
    NA(n->rp, s.nvec * 8);
    NA(n->cvec, s.nvec * 8);
    NA(n->rpp, s.nvec * 8);
#undef NA
    if ((e = hipHostMalloc((void**)&n->h_pinned, 64 * sizeof(double), hipHostMallocDefault)) != hipSuccess) {
        net_destroy(n);
        return e;
    }
    n->g.band = n->band;
    if ((e = hipMemcpy(n->band, s.band.data(), n->g.M * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(n->static_feat, s.static_feat.data(), n->g.M * 8, hipMemcpyHostToDevice)) != hipSuccess) {
        net_destroy(n);
        return e;
    }
    for (uint16_t* a : {n->act0, n->act1, n->act2, n->dz1, n->dz2, n->dy})
        (void)a;
    if ((e = hipMemset(n->act0, 0, s.N * NET_CIN * 2)) != hipSuccess || (e = hipMemset(n->act1, 0, s.N * NET_CH * 2)) != hipSuccess ||
        (e = hipMemset(n->act2, 0, s.N * NET_CH * 2)) != hipSuccess || (e = hipMemset(n->dz1, 0, s.N * NET_CH * 2)) != hipSuccess ||
        (e = hipMemset(n->dz2, 0, s.N * NET_CH * 2)) != hipSuccess || (e = hipMemset(n->dy, 0, s.N * NET_COUT * 2)) != hipSuccess) {
        net_destroy(n);
        return e;
    }
    *out = n;
    return hipSuccess;
}

void net_destroy(NetImpl* n) {
    if (!n) return;
    for (void* q : n->allocs) (void)hipFree(q);
    if (n->h_pinned) (void)hipHostFree(n->h_pinned);
    delete n;
}

int64_t net_band_size(const NetImpl* n) { return n->g.M; }
int64_t net_num_params(const NetImpl* n) { return n->nparams; }
hipError_t net_copy_band(const NetImpl* n, int32_t* host) {
    return hipMemcpy(host, n->band, n->g.M * 4, hipMemcpyDeviceToHost);
}

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t net_set_weights(NetImpl* n, const float* w, hipStream_t s) {
    const float* W1 = w;
    const float* W2 = W1 + 16 * 8 * 27;
    const float* W3 = W2 + 16 * 16 * 27;
    hipLaunchKernelGGL((k_swizzle<8, 16>), dim3(nb256(kc_of(8) * 256)), dim3(256), 0, s, W1, n->wB[0], 0);
    hipLaunchKernelGGL((k_swizzle<16, 16>), dim3(nb256(kc_of(16) * 256)), dim3(256), 0, s, W2, n->wB[1], 0);
    hipLaunchKernelGGL((k_swizzle<16, 4>), dim3(nb256(kc_of(16) * 256)), dim3(256), 0, s, W3, n->wB[2], 0);
    hipLaunchKernelGGL((k_swizzle<16, 16>), dim3(nb256(kc_of(16) * 256)), dim3(256), 0, s, W2, n->wF[1], 1);
    hipLaunchKernelGGL((k_swizzle<16, 4>), dim3(nb256(kc_of(4) * 256)), dim3(256), 0, s, W3, n->wF[2], 1);
    n->weights_set = true;
    return hipGetLastError();
}

hipError_t net_features(NetImpl* n, const double* r, double* scales_host, hipStream_t s) {
    const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n->g.M + 255) / 256));
    hipLaunchKernelGGL(k_band_sumsq, dim3(nblk), dim3(256), 0, s, n->g, r, n->dpartial);
    hipLaunchKernelGGL(k_band_scales, dim3(1), dim3(64), 0, s, n->dpartial, nblk, n->g.M, n->scales);
    hipLaunchKernelGGL(k_band_features, dim3(nb256(n->g.M)), dim3(256), 0, s, n->g, r, n->scales, n->static_feat, n->act0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !scales_host) return e;
    if ((e = hipMemcpyAsync(n->h_pinned, n->scales, 2 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    scales_host[0] = n->h_pinned[0];
    scales_host[1] = n->h_pinned[1];
    return hipSuccess;
}

hipError_t net_forward(NetImpl* n, float* y_out, hipStream_t s) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, (n->g.M + 63) / 64);
    hipLaunchKernelGGL((k_conv<8, 16, 0>), dim3(grid), dim3(256), 0, s, n->g, n->act0, n->wB[0], n->act1, nullptr, nullptr);
    hipLaunchKernelGGL((k_conv<16, 16, 0>), dim3(grid), dim3(256), 0, s, n->g, n->act1, n->wB[1], n->act2, nullptr, nullptr);
    hipLaunchKernelGGL((k_conv<16, 4, 1>), dim3(grid), dim3(256), 0, s, n->g, n->act2, n->wB[2], nullptr, n->y, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && y_out)
        e = hipMemcpyAsync(y_out, n->y, n->g.M * 4 * sizeof(float), hipMemcpyDeviceToDevice, s);
    return e;
}

hipError_t net_targets(NetImpl* n, const double* err, float* t, hipStream_t s) {
    hipLaunchKernelGGL(k_band_targets, dim3(nb256(n->g.M)), dim3(256), 0, s, n->g, err, n->scales, n->static_feat, t);
    return hipGetLastError();
}

hipError_t net_output_grad(NetImpl* n, const double* dldc, double factor, hipStream_t s) {
    hipLaunchKernelGGL(k_band_output_grad, dim3(nb256(n->g.M)), dim3(256), 0, s, n->g, dldc, factor, n->scales,
                       n->static_feat, n->dy);
    return hipGetLastError();
}

hipError_t net_backward(NetImpl* n, const float* t, float* grad, double* loss_host, hipStream_t s) {
    const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n->g.M + 255) / 256));
    if (t) {
        hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, n->g, n->y, t, n->dy, n->dpartial);
        hipLaunchKernelGGL(k_sum_partial, dim3(1), dim3(64), 0, s, n->dpartial, nblk, n->dloss);
    } else {
        loss_host = nullptr;     // dL/dy was supplied by net_output_grad
    }
    const unsigned grid = (unsigned)std::max<int64_t>(1, (n->g.M + 63) / 64);
    float* g1 = grad;
    float* g2 = g1 + 16 * 8 * 27;
    float* g3 = g2 + 16 * 16 * 27;
    const unsigned wb = (unsigned)n->wblocks;
    // layer 3: dW3 from dy and act2; dz2 = (W3^T * dy) masked by relu'(z2)
    hipLaunchKernelGGL((k_wgrad<16, 4>), dim3(wb, (unsigned)((kc_of(16) + 3) / 4)), dim3(256), 0, s, n->g, n->dy, n->act2, n->partial, n->m_per_block);
    hipLaunchKernelGGL(k_sum_blocks, dim3(nb256(4 * 16 * 27)), dim3(256), 0, s, n->partial, (int)wb, (int64_t)(4 * 16 * 27), g3);
    hipLaunchKernelGGL((k_conv<4, 16, 2>), dim3(grid), dim3(256), 0, s, n->g, n->dy, n->wF[2], n->dz2, nullptr, n->act2);
    // layer 2
    hipLaunchKernelGGL((k_wgrad<16, 16>), dim3(wb, (unsigned)((kc_of(16) + 3) / 4)), dim3(256), 0, s, n->g, n->dz2, n->act1, n->partial, n->m_per_block);
    hipLaunchKernelGGL(k_sum_blocks, dim3(nb256(16 * 16 * 27)), dim3(256), 0, s, n->partial, (int)wb, (int64_t)(16 * 16 * 27), g2);
    hipLaunchKernelGGL((k_conv<16, 16, 2>), dim3(grid), dim3(256), 0, s, n->g, n->dz2, n->wF[1], n->dz1, nullptr, n->act1);
    // layer 1
    hipLaunchKernelGGL((k_wgrad<8, 16>), dim3(wb, (unsigned)((kc_of(8) + 3) / 4)), dim3(256), 0, s, n->g, n->dz1, n->act0, n->partial, n->m_per_block);
    hipLaunchKernelGGL(k_sum_blocks, dim3(nb256(16 * 8 * 27)), dim3(256), 0, s, n->partial, (int)wb, (int64_t)(16 * 8 * 27), g1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss_host) return e;
    if ((e = hipMemcpyAsync(n->h_pinned, n->dloss, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *loss_host = n->h_pinned[0];
    return hipSuccess;
}

hipError_t net_adam(int64_t count, float* w, float* m, float* v, const float* g, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nb256(count)), dim3(256), 0, s, count, w, m, v, g, lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

// c = correction from the residual r (dense FP64), written into the dense
// vector c (zeroed first, band entries set)
hipError_t net_output_correction(NetImpl* n, double* c, int64_t nvec, hipStream_t s) {
    hipLaunchKernelGGL((k_zero<double>), dim3(nb256(nvec)), dim3(256), 0, s, c, nvec);
    hipLaunchKernelGGL(k_band_correct, dim3(nb256(n->g.M)), dim3(256), 0, s, n->g, n->y, n->scales, n->static_feat, c);
    return hipGetLastError();
}

hipError_t net_correction(NetImpl* n, const double* r, double* c, int64_t nvec, hipStream_t s) {
    hipError_t e;
    if ((e = net_features(n, r, nullptr, s)) != hipSuccess) return e;
    if ((e = net_forward(n, nullptr, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_zero<double>), dim3(nb256(nvec)), dim3(256), 0, s, c, nvec);
    hipLaunchKernelGGL(k_band_correct, dim3(nb256(n->g.M)), dim3(256), 0, s, n->g, n->y, n->scales, n->static_feat, c);
    return hipGetLastError();
}

hipError_t net_save_input(NetImpl* n, uint16_t* dst, hipStream_t s) {
    hipLaunchKernelGGL((k_band_rows<true>), dim3(nb256(n->g.M * NET_CIN)), dim3(256), 0, s, n->band, n->g.M, n->act0,
                       dst);
    return hipGetLastError();
}

hipError_t net_load_input(NetImpl* n, const uint16_t* src, hipStream_t s) {
    hipLaunchKernelGGL((k_band_rows<false>), dim3(nb256(n->g.M * NET_CIN)), dim3(256), 0, s, n->band, n->g.M, n->act0,
                       const_cast<uint16_t*>(src));
    return hipGetLastError();
}

double* net_work(NetImpl* n, int which) { return which == 0 ? n->rp : which == 1 ? n->cvec : n->rpp; }

}  // namespace iss
