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
// rows and fluxes run one element per thread (the d+1 velocity reads of an
// element are shared by its neighbours through the caches); the B0^T rows one
// vertex per thread over its incident elements.  Every kernel is bound by
// memory traffic.
#include <hip/hip_runtime.h>

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

__constant__ P0Tab g_p0_3 = make_p0tab<3>();
__constant__ P0Tab g_p0_2 = make_p0tab<2>();

template <int D>
__device__ __forceinline__ const P0Tab& p0tab() {
    if constexpr (D == 3) return g_p0_3;
    else return g_p0_2;
}

constexpr double factorial(int d) { return d == 3 ? 6.0 : 2.0; }

// cell coordinates and type of element e
template <int D>
__device__ __forceinline__ void elem_cell(int n, int64_t e, int (&c)[3], int& ty) {
    constexpr int NT = KuhnTables<D>::NT;
    const int64_t cell = e / NT;
    ty = (int)(e - cell * NT);
    c[0] = (int)(cell % n);
    c[1] = (int)((cell / n) % n);
    c[2] = (D == 3) ? (int)(cell / ((int64_t)n * n)) : 0;
}

// the penalty terms w / mu (p_T - p_T') of the facets of element e (zero on
// boundary facets and on facets to an element of another viscosity)
template <int D>
__device__ __forceinline__ void penalty(const LevelView& L, const uint8_t* __restrict__ eph, double w,
                                        const double* __restrict__ p, int64_t e, const int (&c)[3], int ty,
                                        double (&out)[D + 1]) {
    constexpr int NT = KuhnTables<D>::NT;
    const P0Tab& T = p0tab<D>();
    const double mu = L.mu64[eph[e]];
    const double pT = p[e];
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        out[a] = 0.0;
        const int x = c[0] + T.fd[ty][a][0], y = c[1] + T.fd[ty][a][1], z = c[2] + T.fd[ty][a][2];
        const bool in = x >= 0 && x < L.n && y >= 0 && y < L.n && (D == 2 || (z >= 0 && z < L.n));
        if (!in) continue;
        const int64_t e2 = ((int64_t)x + (int64_t)L.n * (y + (int64_t)L.n * (D == 3 ? z : 0))) * NT + T.ft[ty][a];
        if (L.mu64[eph[e2]] == mu) out[a] = w / mu * (pT - p[e2]);
    }
}

// lattice index of vertex a of element (c, ty)
template <int D>
__device__ __forceinline__ int64_t elem_vertex(const LevelView& L, const P0Tab& T, const int (&c)[3], int ty, int a) {
    return (c[0] + T.tv[ty][a][0]) + (int64_t)(c[1] + T.tv[ty][a][1]) * L.sy + (int64_t)(c[2] + T.tv[ty][a][2]) * L.sz;
}

}  // namespace

template <int D>
__global__ __launch_bounds__(256) void k_p0_rows(LevelView L, const uint8_t* __restrict__ eph, double w,
                                                 const double* __restrict__ x, double* __restrict__ y) {
    constexpr int NT = KuhnTables<D>::NT;
    const int n = L.n;
    const int64_t ne = (D == 3 ? (int64_t)n * n * n : (int64_t)n * n) * NT;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const P0Tab& T = p0tab<D>();
    int c[3], ty;
    elem_cell<D>(n, e, c, ty);
    const double* p = x + (int64_t)D * L.N;
    double bu = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        const int64_t v = elem_vertex<D>(L, T, c, ty, a);
#pragma unroll
        for (int l = 0; l < D; ++l) bu += T.g[ty][a][l] * x[(int64_t)l * L.N + v];
    }
    double pen[D + 1];
    penalty<D>(L, eph, w, p, e, c, ty, pen);
    double cp = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a) cp += pen[a];
    y[(int64_t)D * L.N + e] = -(L.sB / factorial(D)) * bu - cp;
}

template <int D>
__global__ __launch_bounds__(256) void k_p0_bt(LevelView L, const double* __restrict__ x, double* __restrict__ y) {
    constexpr int NT = KuhnTables<D>::NT, NS = KuhnTables<D>::NS;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= L.N) return;
    const int n1 = L.n + 1;
    int ijk[3] = {(int)(v % n1), (int)((v / n1) % n1), D == 3 ? (int)(v / ((int64_t)n1 * n1)) : 0};
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

template <int D>
__global__ __launch_bounds__(256) void k_p0_flux(LevelView L, const uint8_t* __restrict__ eph, double w,
                                                 const double* __restrict__ x, double* __restrict__ flux) {
    constexpr int NT = KuhnTables<D>::NT;
    const int n = L.n;
    const int64_t ne = (D == 3 ? (int64_t)n * n * n : (int64_t)n * n) * NT;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const P0Tab& T = p0tab<D>();
    int c[3], ty;
    elem_cell<D>(n, e, c, ty);
    double U[D + 1][D], S[D];
#pragma unroll
    for (int l = 0; l < D; ++l) S[l] = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        const int64_t v = elem_vertex<D>(L, T, c, ty, a);
#pragma unroll
        for (int l = 0; l < D; ++l) {
            U[a][l] = x[(int64_t)l * L.N + v];
            S[l] += U[a][l];
        }
    }
    double pen[D + 1];
    penalty<D>(L, eph, w, x + (int64_t)D * L.N, e, c, ty, pen);
    const double s = -(L.sB / factorial(D));
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        // int_F u_h . n_T = -|T| grad(lambda_a) . sum_{b != a} u_b
        double dot = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) dot += T.g[ty][a][l] * (S[l] - U[a][l]);
        flux[e * (D + 1) + a] = s * dot + pen[a];
    }
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
        hipLaunchKernelGGL(k_p0_bt<3>, dim3(blocks_of(L.N)), dim3(256), 0, s, L, x, y);
        hipLaunchKernelGGL(k_p0_rows<3>, dim3(blocks_of(ne)), dim3(256), 0, s, L, eph, w, x, y);
    } else {
        hipLaunchKernelGGL(k_p0_bt<2>, dim3(blocks_of(L.N)), dim3(256), 0, s, L, x, y);
        hipLaunchKernelGGL(k_p0_rows<2>, dim3(blocks_of(ne)), dim3(256), 0, s, L, eph, w, x, y);
    }
    return hipGetLastError();
}

hipError_t k_p1p0_flux(const LevelView& L, const uint8_t* eph, double gamma, const double* x, double* flux,
                       hipStream_t s) {
    const int D = L.dim;
    const int64_t ne = (D == 3 ? (int64_t)L.n * L.n * L.n * 6 : (int64_t)L.n * L.n * 2);
    const double vol = (D == 3 ? 1.0 / ((double)L.n * L.n * L.n * 6.0) : 1.0 / ((double)L.n * L.n * 2.0));
    const double w = gamma * vol / 4.0;
    if (D == 3) hipLaunchKernelGGL(k_p0_flux<3>, dim3(blocks_of(ne)), dim3(256), 0, s, L, eph, w, x, flux);
    else hipLaunchKernelGGL(k_p0_flux<2>, dim3(blocks_of(ne)), dim3(256), 0, s, L, eph, w, x, flux);
    return hipGetLastError();
}

}  // namespace iss
