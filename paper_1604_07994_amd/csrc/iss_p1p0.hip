// Stabilised P1-P0 operator (Sec. 3): P1 velocity on the lattice vertices,
// piecewise constant pressure on the Kuhn elements (element e = cell * d! +
// type), the interior-penalty stabilisation of eq. stabc and the local flux
// post-process.  System K = [[A, B0^T], [B0, -C]]:
//   (B0 u)_T = -(div u, 1)_T = -|T| sum_a grad(lambda_a) . u_a,
//   (C p)_T  = sum over the facets F of T shared with an element T' of equal
//              viscosity of gamma / (2 mu) |T||T'| / (|T| + |T'|) (p_T - p_T')
//              (no penalty across the interface or on the boundary),
// and the flux of facet F of T is int_F u_h . n_T plus that facet's term of
// (C p)_T, so that the fluxes of an element sum to -(B0 u - C p)_T.
//
// On the lattice every barycentric gradient is an integer vector over h and
// every element has |T| = h^d / d!, so the element terms are compile-time
// integer weights times h^(d-1) / d!.  The element across each facet of a
// type is a fixed (cell offset, type) pair, found at compile time.  Pressure
// rows and fluxes run one cell (d! elements) per thread; the B0^T rows one
// vertex per thread over its incident elements.  Every kernel is bound by
// memory traffic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "iss_internal.h"

namespace iss {

namespace {

template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1, N>(fn);
    }
}

// per element type: vertex offsets, integer barycentric gradients (times h)
// and, per facet (opposite vertex a), the cell offset and type of the
// element across it
struct P0Tab {
    int tv[6][4][3];
    int g[6][4][3];
    int fd[6][4][3];
    int ft[6][4];
};

template <int D>
constexpr P0Tab make_p0tab() {
    constexpr int NT = KuhnTables<D>::NT;
    P0Tab f{};
    for (int ty = 0; ty < NT; ++ty)
        for (int a = 0; a <= D; ++a)
            for (int c = 0; c < 3; ++c) {
                f.tv[ty][a][c] = Kuhn<D>::T.type_vert[ty][a][c];
                f.g[ty][a][c] = c < D ? KGrad<D>::G.g[ty][a][c] : 0;
            }
    for (int ty = 0; ty < NT; ++ty)
        for (int a = 0; a <= D; ++a) {
            int fv[D][3] = {};
            int k = 0;
            for (int b = 0; b <= D; ++b)
                if (b != a) {
                    for (int c = 0; c < 3; ++c) fv[k][c] = f.tv[ty][b][c];
                    ++k;
                }
            for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx)
                        for (int t2 = 0; t2 < NT; ++t2) {
                            if (dx == 0 && dy == 0 && dz == 0 && t2 == ty) continue;
                            int hit = 0;
                            for (int q = 0; q < D; ++q)
                                for (int b2 = 0; b2 <= D; ++b2)
                                    if (f.tv[t2][b2][0] + dx == fv[q][0] && f.tv[t2][b2][1] + dy == fv[q][1] &&
                                        f.tv[t2][b2][2] + dz == fv[q][2])
                                        ++hit;
                            if (hit == D) {
                                f.fd[ty][a][0] = dx;
                                f.fd[ty][a][1] = dy;
                                f.fd[ty][a][2] = dz;
                                f.ft[ty][a] = t2;
                            }
                        }
        }
    return f;
}

// the tables as compile-time constants (indexed only inside unrolled loops)
template <int D> struct P0T { static constexpr P0Tab T = make_p0tab<D>(); };

constexpr double factorial(int d) { return d == 3 ? 6.0 : 2.0; }

}  // namespace

// One thread per cell: the 2^d corner velocities, the cell's d! pressures
// and phases are loaded once and serve all d! element rows; of the facets,
// those inside the cell pair two of its own elements, the others reach the
// element of a neighbouring cell (one pressure and one phase load each).
template <int D>
__device__ __forceinline__ void cell_coords(int n, uint32_t cell, int (&c)[3]) {
    const uint32_t un = (uint32_t)n;
    const uint32_t r = cell / un;
    c[0] = (int)(cell - r * un);
    if (D == 3) {
        const uint32_t r2 = r / un;
        c[1] = (int)(r - r2 * un);
        c[2] = (int)r2;
    } else {
        c[1] = (int)r;
        c[2] = 0;
    }
}

// corner velocities U[corner][l], corner = dx + 2 dy + 4 dz
template <int D>
__device__ __forceinline__ void load_corners(const LevelView& L, const double* __restrict__ x, const int (&c)[3],
                                             double (&U)[1 << D][D]) {
    const int64_t v0 = c[0] + (int64_t)c[1] * L.sy + (int64_t)c[2] * L.sz;
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
        const int64_t v = v0 + (k & 1) + ((k >> 1) & 1) * L.sy + (D == 3 ? ((k >> 2) & 1) * L.sz : 0);
#pragma unroll
        for (int l = 0; l < D; ++l) U[k][l] = x[(int64_t)l * L.N + v];
    }
}

// penalty terms of every facet of the cell's elements: pen[t][a]
template <int D>
__device__ __forceinline__ void cell_penalty(const LevelView& L, const uint8_t* __restrict__ eph, double w,
                                             const double* __restrict__ p, uint32_t cell, const int (&c)[3],
                                             double (&pen)[KuhnTables<D>::NT][D + 1]) {
    constexpr int NT = KuhnTables<D>::NT;
    const int64_t base = (int64_t)cell * NT;
    double P[NT], mu[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        P[t] = p[base + t];
        mu[t] = L.mu64[eph[base + t]];
    }
    static_for<0, NT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        static_for<0, D + 1>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int dx = P0T<D>::T.fd[t][a][0], dy = P0T<D>::T.fd[t][a][1], dz = P0T<D>::T.fd[t][a][2];
            constexpr int t2 = P0T<D>::T.ft[t][a];
            double pn, mun;
            bool in = true;
            if constexpr (dx == 0 && dy == 0 && dz == 0) {
                pn = P[t2];
                mun = mu[t2];
            } else {
                const int x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
                in = x >= 0 && x < L.n && y >= 0 && y < L.n && (D == 2 || (z >= 0 && z < L.n));
                const int64_t e2 = in ? base + ((int64_t)dx + (int64_t)dy * L.n + (int64_t)dz * L.n * L.n) * NT + t2
                                      : base;
                pn = p[e2];
                mun = L.mu64[eph[e2]];
            }
            pen[t][a] = (in && mun == mu[t]) ? w / mu[t] * (P[t] - pn) : 0.0;
        });
    });
}

template <int D>
__global__ __launch_bounds__(256) void k_p0_rows(LevelView L, const uint8_t* __restrict__ eph, double w,
                                                 const double* __restrict__ x, double* __restrict__ y) {
    constexpr int NT = KuhnTables<D>::NT;
    __shared__ double out[256 * NT];
    const int n = L.n;
    const uint32_t ncell = D == 3 ? (uint32_t)n * n * n : (uint32_t)n * n;
    const uint32_t cell0 = blockIdx.x * 256u + threadIdx.x;
    // threads past the last cell compute cell 0 again and do not store it
    const uint32_t cell = cell0 < ncell ? cell0 : 0u;
    int c[3];
    cell_coords<D>(n, cell, c);
    double U[1 << D][D];
    load_corners<D>(L, x, c, U);
    double pen[NT][D + 1];
    cell_penalty<D>(L, eph, w, x + (int64_t)D * L.N, cell, c, pen);
    const double s = -(L.sB / factorial(D));
    static_for<0, NT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        double bu = 0.0, cp = 0.0;
        static_for<0, D + 1>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int k = P0T<D>::T.tv[t][a][0] + 2 * P0T<D>::T.tv[t][a][1] + 4 * P0T<D>::T.tv[t][a][2];
            static_for<0, D>([&](auto lc) {
                constexpr int l = decltype(lc)::value;
                constexpr int g = P0T<D>::T.g[t][a][l];
                if constexpr (g != 0) bu += (double)g * U[k][l];
            });
            cp += pen[t][a];
        });
        out[threadIdx.x * NT + t] = s * bu - cp;
    });
    // the workgroup's rows are contiguous: store them with unit stride
    __syncthreads();
    double* yp = y + (int64_t)D * L.N + (int64_t)blockIdx.x * 256 * NT;
    const uint32_t lim = (ncell - blockIdx.x * 256u < 256u ? ncell - blockIdx.x * 256u : 256u) * NT;
    for (uint32_t q = threadIdx.x; q < lim; q += 256) yp[q] = out[q];
}

template <int D>
__global__ __launch_bounds__(256) void k_p0_bt(LevelView L, const double* __restrict__ x, double* __restrict__ y) {
    constexpr int NT = KuhnTables<D>::NT, NS = KuhnTables<D>::NS;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= L.N) return;
    const uint32_t n1 = (uint32_t)L.n + 1u, uv = (uint32_t)v;
    const uint32_t r = uv / n1;
    int ijk[3] = {(int)(uv - r * n1), D == 3 ? (int)(r - (r / n1) * n1) : (int)r, D == 3 ? (int)(r / n1) : 0};
    const double* p = x + (int64_t)D * L.N;
    double acc[D];
#pragma unroll
    for (int l = 0; l < D; ++l) acc[l] = 0.0;
    static_for<0, NS>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        int cc[3] = {0, 0, 0};
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            cc[a] = ijk[a] + Kuhn<D>::T.slot_cell[sl][a];
            in = in && cc[a] >= 0 && cc[a] < L.n;
        }
        if (!in) return;
        constexpr int ty = Kuhn<D>::T.slot_type[sl], a = Kuhn<D>::T.slot_loc[sl];
        const int64_t e = ((int64_t)cc[0] + (int64_t)L.n * (cc[1] + (int64_t)L.n * (D == 3 ? cc[2] : 0))) * NT + ty;
        const double pe = p[e];
        static_for<0, D>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            constexpr int g = KGrad<D>::G.g[ty][a][l];
            if constexpr (g != 0) acc[l] += (double)g * pe;
        });
    });
    bool bnd = false;
#pragma unroll
    for (int a = 0; a < D; ++a) bnd = bnd || ijk[a] == 0 || ijk[a] == L.n;
    const double s = -(L.sB / factorial(D));
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const bool fixed = L.freeslip ? (ijk[l] == 0 || ijk[l] == L.n) : bnd;
        if (!fixed) y[(int64_t)l * L.N + v] += s * acc[l];
    }
}

// B0^T rows in 3D: a workgroup owns a 64 x 4 tile of vertices and marches
// through a chunk of planes; the pressures of the cells around the tile
// (65 x 5 cells, two cell planes: below and above the vertex plane) sit in
// LDS, loaded with unit-stride reads (a row of cells is contiguous, cell
// major and type minor), so every element pressure comes from memory about
// once instead of once per incident vertex.
constexpr int BT_X = 64, BT_Y = 4, BC_X = BT_X + 1, BC_Y = BT_Y + 1, BC_ROW = BC_X * 6;

__global__ __launch_bounds__(256) void k_p0_bt_z(LevelView L, int zc, const double* __restrict__ x,
                                                 double* __restrict__ y) {
    constexpr int D = 3, NT = 6, NS = KuhnTables<3>::NS;
    __shared__ double lds[2][BC_Y][BC_ROW];
    const int n = L.n;
    const int gx = (n + BT_X) / BT_X, gy = (n + BT_Y) / BT_Y;     // tiles over vertices 0..n
    const int b = (int)blockIdx.x;
    const int tx = b % gx, r = b / gx, tyl = r % gy, tz = r / gy;
    const int i0 = tx * BT_X, j0 = tyl * BT_Y, k0 = tz * zc;
    if (k0 > n) return;                                             // uniform over the workgroup
    const int k1 = min(k0 + zc, n + 1);
    const double* p = x + (int64_t)D * L.N;
    auto load_plane = [&](int ck, int slot) {
        for (int q = (int)threadIdx.x; q < BC_Y * BC_ROW; q += 256) {
            const int row = q / BC_ROW, rem = q - row * BC_ROW;
            const int cc = rem / NT, t = rem - cc * NT;
            const int ci = i0 - 1 + cc, cj = j0 - 1 + row;
            const bool in = ci >= 0 && ci < n && cj >= 0 && cj < n && ck >= 0 && ck < n;
            const int64_t e = in ? (((int64_t)ck * n + cj) * n + ci) * NT + t : 0;
            const double v = p[e];
            lds[slot][row][rem] = in ? v : 0.0;
        }
    };
    load_plane(k0 - 1, 0);
    load_plane(k0, 1);
    __syncthreads();
    int sm = 0, s0 = 1;                                             // cell planes k-1 and k
    const int li = (int)threadIdx.x & (BT_X - 1), lj = (int)threadIdx.x / BT_X;
    const int i = i0 + li, j = j0 + lj;
    const double s = -(L.sB / factorial(D));
    for (int k = k0; k < k1; ++k) {
        if (i <= n && j <= n) {
            double acc[D] = {0.0, 0.0, 0.0};
            static_for<0, NS>([&](auto sc) {
                constexpr int sl = decltype(sc)::value;
                constexpr int sx = Kuhn<3>::T.slot_cell[sl][0], sy = Kuhn<3>::T.slot_cell[sl][1],
                              sz = Kuhn<3>::T.slot_cell[sl][2];
                constexpr int ty = Kuhn<3>::T.slot_type[sl], a = Kuhn<3>::T.slot_loc[sl];
                const double pe = lds[sz < 0 ? sm : s0][lj + 1 + sy][(li + 1 + sx) * NT + ty];
                static_for<0, D>([&](auto lc) {
                    constexpr int l = decltype(lc)::value;
                    constexpr int g = KGrad<3>::G.g[ty][a][l];
                    if constexpr (g != 0) acc[l] += (double)g * pe;
                });
            });
            const int ijk[3] = {i, j, k};
            const bool bnd = i == 0 || i == n || j == 0 || j == n || k == 0 || k == n;
            const int64_t v = i + (int64_t)j * L.sy + (int64_t)k * L.sz;
#pragma unroll
            for (int l = 0; l < D; ++l) {
                const bool fixed = L.freeslip ? (ijk[l] == 0 || ijk[l] == n) : bnd;
                if (!fixed) y[(int64_t)l * L.N + v] += s * acc[l];
            }
        }
        __syncthreads();
        if (k + 1 < k1) load_plane(k + 1, sm);
        __syncthreads();
        const int t = sm;
        sm = s0;
        s0 = t;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_p0_flux(LevelView L, const uint8_t* __restrict__ eph, double w,
                                                 const double* __restrict__ x, double* __restrict__ flux) {
    constexpr int NT = KuhnTables<D>::NT, W = NT * (D + 1);
    __shared__ double out[256 * W];
    const int n = L.n;
    const uint32_t ncell = D == 3 ? (uint32_t)n * n * n : (uint32_t)n * n;
    const uint32_t cell0 = blockIdx.x * 256u + threadIdx.x;
    const uint32_t cell = cell0 < ncell ? cell0 : 0u;
    int c[3];
    cell_coords<D>(n, cell, c);
    double U[1 << D][D];
    load_corners<D>(L, x, c, U);
    double pen[NT][D + 1];
    cell_penalty<D>(L, eph, w, x + (int64_t)D * L.N, cell, c, pen);
    const double s = -(L.sB / factorial(D));
    static_for<0, NT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        static_for<0, D + 1>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            // int_F u_h . n_T = -|T| grad(lambda_a) . sum_{b != a} u_b
            double dot = 0.0;
            static_for<0, D + 1>([&](auto bc) {
                constexpr int b = decltype(bc)::value;
                if constexpr (b != a) {
                    constexpr int k = P0T<D>::T.tv[t][b][0] + 2 * P0T<D>::T.tv[t][b][1] + 4 * P0T<D>::T.tv[t][b][2];
                    static_for<0, D>([&](auto lc) {
                        constexpr int l = decltype(lc)::value;
                        constexpr int g = P0T<D>::T.g[t][a][l];
                        if constexpr (g != 0) dot += (double)g * U[k][l];
                    });
                }
            });
            out[threadIdx.x * W + t * (D + 1) + a] = s * dot + pen[t][a];
        });
    });
    __syncthreads();
    double* fp = flux + (int64_t)blockIdx.x * 256 * W;
    const uint32_t lim = (ncell - blockIdx.x * 256u < 256u ? ncell - blockIdx.x * 256u : 256u) * W;
    for (uint32_t q = threadIdx.x; q < lim; q += 256) fp[q] = out[q];
}

static inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t k_p1p0_apply(const LevelView& L, int form, const uint8_t* eph, double gamma, const double* x, double* y,
                        hipStream_t s) {
    const int D = L.dim;
    const int64_t ne = (D == 3 ? (int64_t)L.n * L.n * L.n * 6 : (int64_t)L.n * L.n * 2);
    const double vol = (D == 3 ? 1.0 / ((double)L.n * L.n * L.n * 6.0) : 1.0 / ((double)L.n * L.n * 2.0));
    // facet weight gamma / (2 mu) |T||T'| / (|T| + |T'|) = gamma |T| / (4 mu)
    const double w = gamma * vol / 4.0;
    hipError_t e = k_apply(L, form, BLOCK_VEL, MODE_APPLY, PREC_F64, x, nullptr, y, s);
    if (e != hipSuccess) return e;
    if (D == 3) {
        const int n = L.n;
        const int gx = (n + BT_X) / BT_X, gy = (n + BT_Y) / BT_Y;
        // z chunks: about four workgroups per CU, at most 32 planes
        const int per_layer = gx * gy;
        const int want = std::max(1, (1024 + per_layer - 1) / per_layer);
        const int zc = std::min(32, std::max(4, (n + 1 + want - 1) / want));
        const int gz = (n + 1 + zc - 1) / zc;
        hipLaunchKernelGGL(k_p0_bt_z, dim3((unsigned)(gx * gy * gz)), dim3(256), 0, s, L, zc, x, y);
        hipLaunchKernelGGL(k_p0_rows<3>, dim3(blocks_of(ne / 6)), dim3(256), 0, s, L, eph, w, x, y);
    } else {
        hipLaunchKernelGGL(k_p0_bt<2>, dim3(blocks_of(L.N)), dim3(256), 0, s, L, x, y);
        hipLaunchKernelGGL(k_p0_rows<2>, dim3(blocks_of(ne / 2)), dim3(256), 0, s, L, eph, w, x, y);
    }
    return hipGetLastError();
}

hipError_t k_p1p0_flux(const LevelView& L, const uint8_t* eph, double gamma, const double* x, double* flux,
                       hipStream_t s) {
    const int D = L.dim;
    const int64_t ne = (D == 3 ? (int64_t)L.n * L.n * L.n * 6 : (int64_t)L.n * L.n * 2);
    const double vol = (D == 3 ? 1.0 / ((double)L.n * L.n * L.n * 6.0) : 1.0 / ((double)L.n * L.n * 2.0));
    const double w = gamma * vol / 4.0;
    if (D == 3) hipLaunchKernelGGL(k_p0_flux<3>, dim3(blocks_of(ne / 6)), dim3(256), 0, s, L, eph, w, x, flux);
    else hipLaunchKernelGGL(k_p0_flux<2>, dim3(blocks_of(ne / 2)), dim3(256), 0, s, L, eph, w, x, flux);
    return hipGetLastError();
}

}  // namespace iss
