// HIP kernels (gfx950) of the matrix-free Stokes hot path.
//
// Operators (Sec. 5 saddle point system K = [[A, B^T], [B, -C]]):
//   * bulk kernels handle interior vertices whose incident elements share
//     one viscosity: constant stencils scaled by that viscosity -- for the
//     gradient and interface forms the decoupled Laplacian stencil per
//     velocity component (eq. equivalence-stencil, Sec. 2.2), for the
//     strain form the coupled 3x3-block stencil (eq. standard);
//   * special kernels handle the compact list of interface and boundary
//     vertices by looping over the incident elements with their own
//     viscosities (the full a_tr / a_sym rows of Sec. 2.2; truncated
//     pressure rows on the boundary).
// The smoother is the Uzawa step of eq. Uzawa_smooth with multicolour
// Gauss-Seidel sweeps; colour (i + j + k) mod (d + 1).  No MFMA: every
// kernel here is bound by HBM traffic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "iss.h"
#include "iss_internal.h"

namespace iss {

__constant__ ElemTables<3, double> g_e3d;
__constant__ ElemTables<3, float> g_e3f;
__constant__ ElemTables<2, double> g_e2d;
__constant__ ElemTables<2, float> g_e2f;

template <int D, typename C> struct ETab;
template <> struct ETab<3, double> { __device__ static const ElemTables<3, double>& get() { return g_e3d; } };
template <> struct ETab<3, float> { __device__ static const ElemTables<3, float>& get() { return g_e3f; } };
template <> struct ETab<2, double> { __device__ static const ElemTables<2, double>& get() { return g_e2d; } };
template <> struct ETab<2, float> { __device__ static const ElemTables<2, float>& get() { return g_e2f; } };

// Arithmetic type of a storage type: BF16-stored vectors are computed in FP32.
template <typename T> struct Acc { using type = T; };
template <> struct Acc<__bf16> { using type = float; };
template <> struct Acc<_Float16> { using type = float; };

template <typename T> struct Prec;
template <> struct Prec<double> {
    __device__ static double mu(const LevelView& L, int ph) { return L.mu64[ph]; }
    __device__ static double imu(const LevelView& L, int ph) { return L.imu64[ph]; }
};
template <> struct Prec<float> {
    __device__ static float mu(const LevelView& L, int ph) { return L.mu32[ph]; }
    __device__ static float imu(const LevelView& L, int ph) { return L.imu32[ph]; }
};

// Table lookup by phase: a wave whose lanes share one phase (the common case
// inside a subdomain) reads the entry once through the scalar cache.
template <typename C>
__device__ __forceinline__ C phase_lookup(const C* __restrict__ tab, int ph) {
    const int p0 = __builtin_amdgcn_readfirstlane(ph);
    if (__all(ph == p0)) return tab[p0];
    return tab[ph];
}

template <typename C> struct PrecU;
template <> struct PrecU<double> {
    __device__ static double mu(const LevelView& L, int ph) { return phase_lookup(L.mu64, ph); }
    __device__ static double imu(const LevelView& L, int ph) { return phase_lookup(L.imu64, ph); }
};
template <> struct PrecU<float> {
    __device__ static float mu(const LevelView& L, int ph) { return phase_lookup(L.mu32, ph); }
    __device__ static float imu(const LevelView& L, int ph) { return phase_lookup(L.imu32, ph); }
};

// ----------------------------------------------------------------------------
// thread -> vertex maps

// Hand the 8 XCDs runs of g consecutive work blocks in turn (used by the
// special-row kernels, whose lists run plane by plane).  The dispatcher
// sends workgroup b to XCD b % 8, so within each stretch of 8 g workgroups
// XCD x takes the blocks [x g, (x + 1) g) of the stretch: rows of
// neighbouring z-planes, a few blocks apart in a list, share most of their
// neighbour lines and now meet in one L2, while every XCD still takes its
// share of every part of the list (boundary rows first, then the more
// costly interior ones).  g = nb / 32 within [2, 16]: 16 on the large
// levels, a few on small grids.  A last stretch shorter than 8 g keeps the
// identity map; the map is a permutation of [0, nb).
__device__ __forceinline__ int64_t xcd_group_remap(int64_t b, int64_t nb) {
    const int64_t g = nb < 64 ? 2 : (nb >= 512 ? 16 : nb >> 5);
    const int64_t span = 8 * g;
    const int64_t st = b / span;
    if ((st + 1) * span > nb) return b;
    const int64_t r = b - st * span;
    return st * span + (r & 7) * g + (r >> 3);
}

// Stencil kernels split the interior rows j = 1..m into 8 slabs of
// ceil(m / 8) rows, one per XCD (workgroup b runs on XCD b % 8), and walk
// each slab in the order x, then y inside the slab, then z.  An XCD then
// works on a narrow band of a few planes at a time, so the rows and planes
// around a vertex are still in its own L2 when they are read again.
constexpr int NXCD = 8;
__device__ __forceinline__ int slab_rows(int m) { return (m + NXCD - 1) / NXCD; }
inline int slab_rows_h(int m) { return (m + NXCD - 1) / NXCD; }

constexpr int BX = 64, BY = 4;   // 256-thread workgroups: 64 along x, 4 rows

// Interior vertex (1..n-1 per axis) of a bulk kernel (64 x 4 tiles inside
// the XCD's slab).  Returns false for threads outside the interior.
template <int D>
__device__ __forceinline__ bool interior_vertex(const LevelView& L, int64_t bid, int& i, int& j, int& k) {
    const int m = L.n - 1;                       // interior points per axis
    const int rows = slab_rows(m);
    const int gx = (m + BX - 1) / BX, gys = (rows + BY - 1) / BY;
    const int xcd = (int)(bid & (NXCD - 1));
    const int64_t idx = bid / NXCD;
    const int bx = (int)(idx % gx);
    const int64_t r = idx / gx;
    const int by = (int)(r % gys);
    k = (D == 3) ? 1 + (int)(r / gys) : 0;
    const int jl = by * BY + (int)threadIdx.y;
    j = 1 + xcd * rows + jl;
    i = 1 + bx * BX + (int)threadIdx.x;
    return jl < rows && j <= m && i <= m && (D == 2 || k <= m);
}

template <int D>
inline int64_t interior_blocks(int n) {
    const int m = n - 1;
    if (m <= 0) return 0;
    const int rows = slab_rows_h(m);
    return (int64_t)NXCD * ((m + BX - 1) / BX) * ((rows + BY - 1) / BY) * (D == 3 ? m : 1);
}

template <int D>
__device__ __forceinline__ int64_t nb_lin(const LevelView& L, int o) {
    constexpr auto& T = Kuhn<D>::T;
    return (int64_t)T.off[o][0] + (int64_t)T.off[o][1] * L.sy + (int64_t)T.off[o][2] * L.sz;
}

// ----------------------------------------------------------------------------
// neighbourhood loads

template <int D, int NF, typename T, typename C>
__device__ __forceinline__ void load_interior(const LevelView& L, const T* __restrict__ x,
                                              int64_t v, int f0, C (&V)[NF][KuhnTables<D>::NB]) {
    constexpr int NB = KuhnTables<D>::NB;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int o = 0; o < NB; ++o)
            V[f][o] = (C)x[(int64_t)(f0 + f) * L.N + v + nb_lin<D>(L, o)];
}

// guarded load for vertices that may sit on the boundary
// compile-time loop: fn(integral_constant<int, i>) for i = I..N-1
template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1, N>(fn);
    }
}

template <int D, int NF, typename T, typename C>
__device__ __forceinline__ void load_guarded(const LevelView& L, const T* __restrict__ x,
                                             int64_t v, const int (&ijk)[3], int f0,
                                             C (&V)[NF][KuhnTables<D>::NB]) {
    static_for<0, KuhnTables<D>::NB>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        constexpr int dx = Kuhn<D>::T.off[o][0], dy = Kuhn<D>::T.off[o][1], dz = Kuhn<D>::T.off[o][2];
        const bool in = (ijk[0] + dx >= 0) && (ijk[0] + dx <= L.n) && (ijk[1] + dy >= 0) &&
                        (ijk[1] + dy <= L.n) && (D == 2 || ((ijk[2] + dz >= 0) && (ijk[2] + dz <= L.n)));
        // unconditional load from a clamped index, then a select: no branch
        const int64_t nv = in ? v + dx + (int64_t)dy * L.sy + (int64_t)dz * L.sz : v;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const C val = (C)x[(int64_t)(f0 + f) * L.N + nv];
            V[f][o] = in ? val : (C)0;
        }
    });
}

// (a lattice has fewer than 2^32 vertices: 32-bit division suffices)
template <int D>
__device__ __forceinline__ void vertex_ijk(const LevelView& L, int64_t v, int (&ijk)[3]) {
    const uint32_t n1 = (uint32_t)L.n + 1u, u = (uint32_t)v;
    const uint32_t r = u / n1;
    ijk[0] = (int)(u - r * n1);
    const uint32_t r2 = r / n1;
    ijk[1] = (int)(r - r2 * n1);
    ijk[2] = (D == 3) ? (int)r2 : 0;
}

template <int D>
__device__ __forceinline__ bool on_boundary(const LevelView& L, const int (&ijk)[3]) {
    bool b = false;
#pragma unroll
    for (int a = 0; a < D; ++a) b = b || ijk[a] == 0 || ijk[a] == L.n;
    return b;
}

// velocity component l of the vertex is fixed (eq. boundary): every
// component of a boundary vertex for no-slip, the normal component on each
// face for free-slip
template <int D>
__device__ __forceinline__ bool vel_fixed(const LevelView& L, const int (&ijk)[3], int l) {
    return L.freeslip ? (ijk[l] == 0 || ijk[l] == L.n) : on_boundary<D>(L, ijk);
}

// ----------------------------------------------------------------------------
// element loop of one special vertex: rows of A (form F), B^T, B and C.

template <int D, int F, bool VEL, bool PRES, typename C>
struct RowAcc {
    C au[D];          // sum_T mu_T A_T u          (unscaled by sA)
    C abt[D];         // sum_T B_T^T p             (unscaled by sB)
    C Dm[D][D];       // point diagonal block of sum_T mu_T A_T
    C bdiv;           // sum_T B_T u
    C cp;             // sum_T (1/mu_T) C_T p      (unscaled by sC)
    C cd;             // sum_T (1/mu_T) C_T delta
    C cjj;            // point diagonal of sum_T (1/mu_T) C_T
};

// The slot, vertex and component loops are unrolled at compile time: every
// index into the preloaded footprint arrays is a constant (registers, no
// scratch), and every element-matrix entry is an integer known at compile
// time (exact Kuhn gradients; the common factors |T| and -|T|/(d+1) are
// applied once at the end), so zero entries cost nothing and no table is
// read.
template <int D, int F, bool VEL, bool PRES, bool WANT_D, bool WANT_DELTA, typename C>
__device__ __forceinline__ void element_rows(const LevelView& L, int64_t s,
                                             const C (&U)[D][KuhnTables<D>::NB],
                                             const C (&P)[KuhnTables<D>::NB],
                                             const C (&Dl)[KuhnTables<D>::NB],
                                             RowAcc<D, F, VEL, PRES, C>& r) {
    constexpr int NS = KuhnTables<D>::NS;
    constexpr C VOL = (C)kuhn_volume<D>();
    constexpr C BVOL = (C)(-kuhn_volume<D>() / (D + 1));
#pragma unroll
    for (int a = 0; a < D; ++a) {
        r.au[a] = 0; r.abt[a] = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) r.Dm[a][b] = 0;
    }
    r.bdiv = 0; r.cp = 0; r.cd = 0; r.cjj = 0;
    // phases of all incident elements first (one batch of loads), then the
    // viscosities; an element outside the domain contributes with weight 0
    int ph[NS];
    {
        const uint8_t* eph = L.spec_eph + s * NS;
        if constexpr (NS % 4 == 0) {
            const uint32_t* e32 = reinterpret_cast<const uint32_t*>(eph);   // 3D: 24 bytes, 8-aligned
#pragma unroll
            for (int q = 0; q < NS / 4; ++q) {
                const uint32_t wd = e32[q];
#pragma unroll
                for (int t = 0; t < 4; ++t) ph[4 * q + t] = (int)((wd >> (8 * t)) & 0xffu);
            }
        } else {
#pragma unroll
            for (int q = 0; q < NS; ++q) ph[q] = eph[q];
        }
    }
    C inw[NS], muv[NS], imuv[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        inw[q] = ph[q] != OUTSIDE ? (C)1 : (C)0;
        if constexpr (VEL) muv[q] = inw[q] * Prec<C>::mu(L, ph[q]);
        if constexpr (PRES) imuv[q] = inw[q] * Prec<C>::imu(L, ph[q]);
    }
    static_for<0, NS>([&](auto slc) {
        constexpr int sl = decltype(slc)::value;
        constexpr int ty = Kuhn<D>::T.slot_type[sl];
        constexpr int a = Kuhn<D>::T.slot_loc[sl];
        if constexpr (VEL) {
            const C mu = muv[sl];
            C au[D], psum = 0;
#pragma unroll
            for (int l = 0; l < D; ++l) au[l] = 0;
            static_for<0, D + 1>([&](auto bc) {
                constexpr int bb = decltype(bc)::value;
                constexpr int o = Kuhn<D>::T.slot_nb[sl][bb];
                psum += P[o];
                static_for<0, D>([&](auto lc) {
                    constexpr int l = decltype(lc)::value;
                    static_for<0, D>([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        constexpr int A = kg_visc<D>(F, ty, a, l, bb, k);
                        if constexpr (A != 0) au[l] += (C)A * U[k][o];
                        if constexpr (WANT_D && bb == a && A != 0) r.Dm[l][k] += mu * (C)A;
                    });
                });
            });
            static_for<0, D>([&](auto lc) {
                constexpr int l = decltype(lc)::value;
                r.au[l] += mu * au[l];
                constexpr int ga = KGrad<D>::G.g[ty][a][l];
                if constexpr (ga != 0) r.abt[l] += (C)ga * (inw[sl] * psum);
            });
        }
        if constexpr (PRES) {
            const C imu = imuv[sl];
            C bd = 0, cp = 0, cd = 0;
            static_for<0, D + 1>([&](auto bc) {
                constexpr int bb = decltype(bc)::value;
                constexpr int o = Kuhn<D>::T.slot_nb[sl][bb];
                static_for<0, D>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    constexpr int gb = KGrad<D>::G.g[ty][bb][k];
                    if constexpr (gb != 0) bd += (C)gb * U[k][o];
                });
                constexpr int cg = kg_dot<D>(ty, a, bb);
                if constexpr (cg != 0) {
                    cp += (C)cg * P[o];
                    if constexpr (WANT_DELTA) cd += (C)cg * Dl[o];
                }
            });
            r.bdiv += inw[sl] * bd;
            r.cp += imu * cp;
            if constexpr (WANT_DELTA) r.cd += imu * cd;
            if constexpr (WANT_D) r.cjj += imu * (C)kg_dot<D>(ty, a, a);
        }
    });
#pragma unroll
    for (int l = 0; l < D; ++l) {
        r.au[l] *= VOL;
        r.abt[l] *= BVOL;
#pragma unroll
        for (int k = 0; k < D; ++k) r.Dm[l][k] *= VOL;
    }
    r.bdiv *= BVOL;
    r.cp *= VOL;
    r.cd *= VOL;
    r.cjj *= VOL;
}

// ----------------------------------------------------------------------------
// operator apply / residual

template <int D, int F, int BLK, int MODE, typename T>
__device__ __forceinline__ void apply_bulk_body(const LevelView& L, int64_t bid, const T* __restrict__ x,
                                                const T* __restrict__ b, T* __restrict__ y) {
    using C = typename Acc<T>::type;
    constexpr int NB = KuhnTables<D>::NB;
    int i, j, k;
    if (!interior_vertex<D>(L, bid, i, j, k)) return;
    const int64_t v = i + j * L.sy + k * L.sz;
    const int ph = L.vphase[v];
    if (ph == SPECIAL) return;
    const auto& E = ETab<D, C>::get();
    const C mu = Prec<C>::mu(L, ph);
    const C smu = mu * (C)L.sA;
    C out[D + 1];
    if (BLK == BLOCK_FULL || F == FORM_STRAIN) {
        C U[D][NB];
        load_interior<D, D, T, C>(L, x, v, 0, U);
        if (F == FORM_STRAIN) {
#pragma unroll
            for (int l = 0; l < D; ++l) {
                C acc = 0;
#pragma unroll
                for (int kk = 0; kk < D; ++kk)
#pragma unroll
                    for (int o = 0; o < NB; ++o) acc += E.Svis[1][l][kk][o] * U[kk][o];
                out[l] = smu * acc;
            }
        } else {
#pragma unroll
            for (int l = 0; l < D; ++l) {
                C acc = E.Svis[0][l][l][0] * U[l][0];
#pragma unroll
                for (int o = 1; o <= 2 * D; ++o) acc += E.Svis[0][l][l][o] * U[l][o];
                out[l] = smu * acc;
            }
        }
        if (BLK == BLOCK_FULL) {
            C P[1][NB];
            load_interior<D, 1, T, C>(L, x, v, D, P);
            const C sB = (C)L.sB;
#pragma unroll
            for (int l = 0; l < D; ++l) {
                C acc = 0;
#pragma unroll
                for (int o = 1; o < NB; ++o) acc += E.Sbt[l][o] * P[0][o];
                out[l] += sB * acc;
            }
            C dv = 0;
#pragma unroll
            for (int kk = 0; kk < D; ++kk)
#pragma unroll
                for (int o = 1; o < NB; ++o) dv += E.Sdiv[kk][o] * U[kk][o];
            C cp = E.Sc[0] * P[0][0];
#pragma unroll
            for (int o = 1; o <= 2 * D; ++o) cp += E.Sc[o] * P[0][o];
            out[D] = sB * dv - (C)L.sC * Prec<C>::imu(L, ph) * cp;
        } else {
            out[D] = 0;
        }
    } else {
        // decoupled Laplacian rows: only the axis neighbours of each component
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const T* ul = x + (int64_t)l * L.N + v;
            C acc = E.Svis[0][l][l][0] * (C)ul[0];
#pragma unroll
            for (int o = 1; o <= 2 * D; ++o) acc += E.Svis[0][l][l][o] * (C)ul[nb_lin<D>(L, o)];
            out[l] = smu * acc;
        }
        out[D] = 0;
    }
#pragma unroll
    for (int f = 0; f <= D; ++f) {
        const int64_t e = (int64_t)f * L.N + v;
        if (MODE == MODE_RESID)
            y[e] = (BLK == BLOCK_FULL || f < D) ? (T)((C)b[e] - out[f]) : (T)0.0f;
        else
            y[e] = (T)out[f];
    }
}

template <int D, int F, int BLK, int MODE, typename T>
__device__ __forceinline__ void apply_special_body(const LevelView& L, int64_t s, const T* __restrict__ x,
                                                   const T* __restrict__ b, T* __restrict__ y) {
    using C = typename Acc<T>::type;
    constexpr int NB = KuhnTables<D>::NB;
    if (s >= L.spec_off[D + 1]) return;
    const int64_t v = L.spec[s];
    int ijk[3];
    vertex_ijk<D>(L, v, ijk);
    if (!L.freeslip && on_boundary<D>(L, ijk)) {
        // no-slip velocity rows are zero; only the (truncated) pressure
        // row of the full operator is formed
        C out[D + 1];
#pragma unroll
        for (int l = 0; l < D; ++l) out[l] = 0;
        out[D] = 0;
        if (BLK == BLOCK_FULL) {
            C U[D][NB], P[1][NB];
            load_guarded<D, D, T, C>(L, x, v, ijk, 0, U);
            load_guarded<D, 1, T, C>(L, x, v, ijk, D, P);
            RowAcc<D, F, false, true, C> r;
            element_rows<D, F, false, true, false, false, C>(L, s, U, P[0], P[0], r);
            out[D] = (C)L.sB * r.bdiv - (C)L.sC * r.cp;
        }
#pragma unroll
        for (int f = 0; f <= D; ++f) {
            const int64_t e = (int64_t)f * L.N + v;
            if (MODE == MODE_RESID)
                y[e] = (f == D && BLK == BLOCK_FULL) ? (T)((C)b[e] - out[f]) : (T)0.0f;
            else
                y[e] = (T)out[f];
        }
        return;
    }
    // interface rows, and free-slip boundary rows (the full rows of the
    // form on Gamma_F, Sec. 2.2) with their normal component fixed
    C U[D][NB], P[1][NB];
    load_guarded<D, D, T, C>(L, x, v, ijk, 0, U);
    load_guarded<D, 1, T, C>(L, x, v, ijk, D, P);
    RowAcc<D, F, true, BLK == BLOCK_FULL, C> r;
    element_rows<D, F, true, BLK == BLOCK_FULL, false, false, C>(L, s, U, P[0], P[0], r);
    bool fix[D];
#pragma unroll
    for (int l = 0; l < D; ++l) fix[l] = vel_fixed<D>(L, ijk, l);
    C out[D + 1];
#pragma unroll
    for (int l = 0; l < D; ++l)
        out[l] = fix[l] ? (C)0 : (C)L.sA * r.au[l] + (BLK == BLOCK_FULL ? (C)L.sB * r.abt[l] : (C)0);
    out[D] = (BLK == BLOCK_FULL) ? (C)L.sB * r.bdiv - (C)L.sC * r.cp : (C)0;
#pragma unroll
    for (int f = 0; f <= D; ++f) {
        const int64_t e = (int64_t)f * L.N + v;
        if (MODE == MODE_RESID) {
            const bool zero = (f < D && fix[f < D ? f : 0]) || (f == D && BLK != BLOCK_FULL);
            y[e] = zero ? (T)0.0f : (T)((C)b[e] - out[f]);
        } else {
            y[e] = (T)out[f];
        }
    }
}

// Applies: one launch over the interior isoviscous vertices (bulk
// stencils), one over the special-vertex list (element loops).

template <int D, int F, int BLK, int MODE, typename T>
__global__ __launch_bounds__(256) void k_apply_bulk(LevelView L, const T* __restrict__ x,
                                                    const T* __restrict__ b, T* __restrict__ y) {
    apply_bulk_body<D, F, BLK, MODE, T>(L, blockIdx.x, x, b, y);
}

template <int D, int F, int BLK, int MODE, typename T>
__global__ __launch_bounds__(256) void k_apply_special(LevelView L, const T* __restrict__ x,
                                                       const T* __restrict__ b, T* __restrict__ y) {
    apply_special_body<D, F, BLK, MODE, T>(L, xcd_group_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x, x, b, y);
}

// ----------------------------------------------------------------------------
// Uzawa smoother in the colour-split layout
//
// During a smoothing call every field lives in a second layout: row by row,
// the vertices of a row grouped by i mod M (M = d + 1 colours),
//     (i, j, k) -> k Pp + j Rp + (i mod M) q + i div M,
// q = ceil((n + 1) / M), Rp = M q, Pp = (n + 1) Rp.  The vertices of colour
// c = (i + j + k) mod M in a row form the single run i mod M = (c - j - k)
// mod M, so a colour phase reads and writes unit-stride runs instead of
// every M-th element.  Row padding (i > n) is written as zero by the pack
// kernel and never touched by the smoother.

template <int D>
__device__ __forceinline__ int64_t sidx(const LevelView& L, int i, int j, int k) {
    constexpr int M = D + 1;
    return (int64_t)k * L.Pp + (int64_t)j * L.Rp + (int64_t)(i % M) * L.q + i / M;
}

// split-layout offsets of the i-1 and i+1 neighbours of a vertex in run s
struct XOff {
    int64_t m, p;
};

template <int D>
__device__ __forceinline__ XOff x_offsets(const LevelView& L, int s) {
    constexpr int M = D + 1;
    XOff o;
    o.m = (s > 0) ? -(int64_t)L.q : (int64_t)(M - 1) * L.q - 1;
    o.p = (s < M - 1) ? (int64_t)L.q : 1 - (int64_t)(M - 1) * L.q;
    return o;
}

template <int D>
__device__ __forceinline__ int64_t snb(const LevelView& L, const XOff& xo, int o) {
    constexpr auto& T = Kuhn<D>::T;
    const int dx = T.off[o][0];
    return (dx < 0 ? xo.m : (dx > 0 ? xo.p : (int64_t)0)) + (int64_t)T.off[o][1] * L.Rp +
           (int64_t)T.off[o][2] * L.Pp;
}

// Split-layout passes: the threads of XCD x cover its slab of interior rows
// with run positions fastest, then rows, then planes.  `per_row` is the
// number of positions per row the pass visits; bid is a 256-thread group and
// tid the thread within it.  Returns false past the end.
template <int D>
__device__ __forceinline__ bool split_slab_thread(const LevelView& L, int64_t bid, int tid, int per_row, int& pos,
                                                  int& j, int& k) {
    const int m = L.n - 1;
    const int rows = slab_rows(m);
    const int xcd = (int)(bid & (NXCD - 1));
    const int64_t g = (bid / NXCD) * 256 + tid;
    pos = (int)(g % per_row);
    const int64_t r = g / per_row;
    const int jl = (int)(r % rows);
    k = (D == 3) ? 1 + (int)(r / rows) : 0;
    j = 1 + xcd * rows + jl;
    return j <= m && (D == 3 ? k <= m : r < rows);
}

template <int D>
inline int64_t split_slab_blocks(int n, int per_row) {
    const int m = n - 1;
    if (m <= 0) return 0;
    const int64_t per_xcd = (int64_t)per_row * slab_rows_h(m) * (D == 3 ? m : 1);
    return NXCD * ((per_xcd + 255) / 256);
}

// colour phase: interior vertex of colour `colour` (run s of its row)
template <int D>
__device__ __forceinline__ bool split_colour_vertex(const LevelView& L, int colour, int64_t bid, int tid, int& s,
                                                    int64_t& v) {
    constexpr int M = D + 1;
    const int m = L.n - 1;
    int t, j, k;
    if (!split_slab_thread<D>(L, bid, tid, m / M + 1, t, j, k)) return false;
    s = (colour - j - k) % M;
    if (s < 0) s += M;
    const int i = M * t + s;
    if (i < 1 || i > m) return false;
    v = (int64_t)k * L.Pp + (int64_t)j * L.Rp + (int64_t)s * L.q + t;
    return true;
}

// all-interior pass: interior vertex at row position r (run s) and its
// colour (i + j + k) mod (d + 1)
template <int D>
__device__ __forceinline__ bool split_all_vertex(const LevelView& L, int64_t bid, int tid, int& s, int64_t& v,
                                                 int& colour) {
    constexpr int M = D + 1;
    const int m = L.n - 1;
    int r, j, k;
    if (!split_slab_thread<D>(L, bid, tid, L.Rp, r, j, k)) return false;
    s = r / L.q;
    const int i = M * (r - s * L.q) + s;
    if (i < 1 || i > m) return false;
    v = (int64_t)k * L.Pp + (int64_t)j * L.Rp + r;
    colour = (i + j + k) % M;
    return true;
}

template <int D, int NF, typename T, typename C>
__device__ __forceinline__ void load_split(const LevelView& L, const T* __restrict__ xs, int64_t v,
                                           const XOff& xo, int f0, C (&V)[NF][KuhnTables<D>::NB]) {
    constexpr int NB = KuhnTables<D>::NB;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int o = 0; o < NB; ++o) V[f][o] = (C)xs[(int64_t)(f0 + f) * L.Ns + v + snb<D>(L, xo, o)];
}

// guarded split-layout loads around a special vertex (may be on the boundary)
template <int D, int NF, typename T, typename C>
__device__ __forceinline__ void load_guarded_split(const LevelView& L, const T* __restrict__ xs,
                                                   const int (&ijk)[3], int f0,
                                                   C (&V)[NF][KuhnTables<D>::NB]) {
    static_for<0, KuhnTables<D>::NB>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        constexpr int dx = Kuhn<D>::T.off[o][0], dy = Kuhn<D>::T.off[o][1], dz = Kuhn<D>::T.off[o][2];
        const bool in = (ijk[0] + dx >= 0) && (ijk[0] + dx <= L.n) && (ijk[1] + dy >= 0) &&
                        (ijk[1] + dy <= L.n) && (D == 2 || ((ijk[2] + dz >= 0) && (ijk[2] + dz <= L.n)));
        // unconditional load from a clamped index, then a select: no branch
        const int64_t e = in ? sidx<D>(L, ijk[0] + dx, ijk[1] + dy, ijk[2] + dz) : (int64_t)0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const C val = (C)xs[(int64_t)(f0 + f) * L.Ns + e];
            V[f][o] = in ? val : (C)0;
        }
    });
}

// canonical (x fastest) <-> colour-split copies of nf fields.  The pack
// walks the split positions (padding included, written as zero); the
// unpack walks the canonical positions.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_pack_t(LevelView L, const T* __restrict__ in, T* __restrict__ out) {
    constexpr int M = D + 1;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = L.Ns;
    if (e >= per) return;
    const int f = blockIdx.y;
    const int64_t row = e / L.Rp;
    const int r = (int)(e - row * L.Rp);
    const int s = r / L.q;
    const int i = M * (r - s * L.q) + s;
    const int64_t n1 = L.n + 1;
    out[(int64_t)f * per + e] = (i <= L.n) ? in[(int64_t)f * L.N + row * n1 + i] : (T)0.0f;
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_unpack_t(LevelView L, const T* __restrict__ in, T* __restrict__ out) {
    constexpr int M = D + 1;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= L.N) return;
    const int f = blockIdx.y;
    const int64_t n1 = L.n + 1;
    const int64_t row = v / n1;
    const int i = (int)(v - row * n1);
    out[(int64_t)f * L.N + v] = in[(int64_t)f * L.Ns + row * L.Rp + (int64_t)(i % M) * L.q + i / M];
}

// Velocity: one colour phase of the symmetric Gauss-Seidel sweep on
// A u = f - B^T p (eq. Uzawa_smooth).  BWD selects the reversed component
// order of the block update.
template <int D, int F, bool BWD, typename C>
__device__ __forceinline__ void block_gs_update(C (&r)[D], const C (&Dm)[D][D], C (&du)[D]) {
    if (!BWD) {
#pragma unroll
        for (int l = 0; l < D; ++l) {
            C rl = r[l];
#pragma unroll
            for (int k = 0; k < l; ++k) rl -= Dm[l][k] * du[k];
            du[l] = rl / Dm[l][l];
        }
    } else {
#pragma unroll
        for (int l = D - 1; l >= 0; --l) {
            C rl = r[l];
#pragma unroll
            for (int k = D - 1; k > l; --k) rl -= Dm[l][k] * du[k];
            du[l] = rl / Dm[l][l];
        }
    }
}

// All-interior right-hand-side passes.  A thread owns position t of every
// run of a row, i.e. the d+1 consecutive vertices i = (d+1) t + s, so one
// coalesced load per run fetches a footprint row for all of them; the x
// neighbours outside the group (i - 1 of s = 0, i + 1 of s = d) come from
// the neighbouring lanes, or from a direct load at row ends and wave edges.
// The stencil weights are the compile-time integer stencils of the Kuhn
// lattice (times -|T|/(d+1) for B and B^T, |T| for C).
template <int D>
__device__ __forceinline__ bool rhs_thread(const LevelView& L, int& t, int& j, int& k, int& tn) {
    const int m = L.n - 1;
    tn = m / (D + 1) + 1;                          // positions covering i = 1..m
    const bool act = split_slab_thread<D>(L, blockIdx.x, threadIdx.x, tn, t, j, k);
    if (!act) {                                    // keep the lane for the shuffles
        j = m;
        k = (D == 3) ? m : 0;
    }
    return act;
}

// v[0] = value at i = (d+1) t - 1, v[1 + s] = run s at t, v[d + 2] = value at
// i = (d+1)(t + 1), for the row starting at split index rb of field f.
// element e of field f through a 32-bit byte offset from the field base (a
// field has far fewer than 2^29 entries), so the loads use a scalar base
// and one 32-bit offset register
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ f, uint32_t e) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(f) + e * (uint32_t)sizeof(T));
}

template <int D, typename T, typename C>
__device__ __forceinline__ void row_runs(const LevelView& L, const T* __restrict__ f, uint32_t rb, int t,
                                         int tn, C (&v)[D + 3]) {
    constexpr int M = D + 1;
    const uint32_t q = (uint32_t)L.q;
#pragma unroll
    for (int r = 0; r < M; ++r) v[1 + r] = (C)ld32(f, rb + (uint32_t)r * q + (uint32_t)t);
    // the two outer neighbours lie in the same cache lines as the runs
    // (shifted by one position), so direct loads cost little
    // (clamped addresses and selects instead of branches)
    const C lv = (C)ld32(f, rb + (uint32_t)(M - 1) * q + (uint32_t)(t > 0 ? t - 1 : 0));
    const C rv = (C)ld32(f, rb + (uint32_t)min(t + 1, L.q - 1));
    v[0] = (t > 0) ? lv : (C)0;
    v[M + 1] = (M * (t + 1) <= L.n) ? rv : (C)0;
    (void)tn;
}

constexpr int ROW_DY[7] = {0, 1, -1, 0, 0, 1, -1};
constexpr int ROW_DZ[7] = {0, 0, 0, 1, -1, 1, -1};
template <int D> constexpr int rhs_rows() { return D == 3 ? 7 : 3; }

// does footprint row (dy, dz) carry a nonzero weight?  KIND 0: B row of
// component c; 1: B^T (any component); 2: C
template <int D, int KIND, int CMP>
constexpr bool row_used(int dy, int dz) {
    for (int dx = -1; dx <= 1; ++dx) {
        const int o = off_index<D>(dx, dy, dz);
        if (o < 0) continue;
        if (KIND == 0 && sdiv_int<D>(CMP, o) != 0) return true;
        if (KIND == 2 && sc_int<D>(o) != 0) return true;
        if (KIND == 1)
            for (int l = 0; l < D; ++l)
                if (sbt_int<D>(l, o) != 0) return true;
    }
    return false;
}

// g = f - B^T p on interior isoviscous vertices (p is fixed during the
// velocity sweep, so the coupling term is formed once per sweep).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_vel_rhs_s(LevelView L, const T* __restrict__ xs,
                                                   const T* __restrict__ bs, T* __restrict__ g) {
    using C = typename Acc<T>::type;
    constexpr int M = D + 1;
    int t, j, k, tn;
    const bool act = rhs_thread<D>(L, t, j, k, tn);
    const int64_t rb0 = (int64_t)k * L.Pp + (int64_t)j * L.Rp;
    C acc[D][M];
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
        for (int q = 0; q < M; ++q) acc[l][q] = 0;
    static_for<0, rhs_rows<D>()>([&](auto rc) {
        constexpr int dy = ROW_DY[decltype(rc)::value];
        constexpr int dz = D == 3 ? ROW_DZ[decltype(rc)::value] : 0;
        constexpr bool used = row_used<D, 1, 0>(dy, dz);
        if constexpr (used) {
            C v[M + 2];
            row_runs<D, T, C>(L, xs + (int64_t)D * L.Ns, (uint32_t)(rb0 + (int64_t)dy * L.Rp + (int64_t)dz * L.Pp), t,
                              tn, v);
            static_for<0, M>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                static_for<0, 3>([&](auto xc) {
                    constexpr int dx = decltype(xc)::value - 1;
                    constexpr int o = off_index<D>(dx, dy, dz);
                    if constexpr (o >= 0) {
                        static_for<0, D>([&](auto lc) {
                            constexpr int l = decltype(lc)::value;
                            constexpr int w = sbt_int<D>(l, o);
                            if constexpr (w != 0) acc[l][q] += (C)w * v[1 + q + dx];
                        });
                    }
                });
            });
        }
    });
    if (!act) return;
    const int m = L.n - 1;
    const C sbv = (C)(L.sB * (-kuhn_volume<D>() / (D + 1)));
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const int i = M * t + q;
        if (i < 1 || i > m) continue;
        const int64_t v = rb0 + (int64_t)q * L.q + t;
        if (L.vphase_s[v] == SPECIAL) continue;
#pragma unroll
        for (int l = 0; l < D; ++l)
            g[(int64_t)l * L.Ns + v] = (T)((C)bs[(int64_t)l * L.Ns + v] - sbv * acc[l][q]);
    }
}

// Grouped s pass for the larger levels: a thread owns position t of every
// run of a row, i.e. the d+1 consecutive vertices i = (d+1) t + q, as in
// k_vel_rhs_s, so one coalesced load per run and footprint row serves all
// of them.  The fields are read and accumulated one after another, so only
// one field's footprint rows are live in registers.  Integer stencils (B times -|T|/(d+1), C times |T|) and the
// colour-0 update of the first pressure phase as in k_p_rhs_s.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_p_rhs_g(LevelView L, const T* __restrict__ xs,
                                                 const T* __restrict__ bs, T* __restrict__ sres,
                                                 T* __restrict__ delta) {
    using C = typename Acc<T>::type;
    constexpr int M = D + 1;
    int t, j, k, tn;
    const bool act = rhs_thread<D>(L, t, j, k, tn);
    const int64_t rb0 = (int64_t)k * L.Pp + (int64_t)j * L.Rp;
    C dv[M], cp[M];
#pragma unroll
    for (int q = 0; q < M; ++q) { dv[q] = 0; cp[q] = 0; }
    // velocity fields: a rolled loop (one field's footprint rows live at a
    // time); the integer weight of component f is a uniform select
#pragma unroll 1
    for (int f = 0; f < D; ++f) {
        static_for<0, rhs_rows<D>()>([&](auto rc) {
            constexpr int dy = ROW_DY[decltype(rc)::value];
            constexpr int dz = D == 3 ? ROW_DZ[decltype(rc)::value] : 0;
            constexpr bool used = row_used<D, 0, 0>(dy, dz) || row_used<D, 0, 1>(dy, dz) ||
                                  (D == 3 && row_used<D, 0, D - 1>(dy, dz));
            if constexpr (used) {
                C v[M + 2];
                row_runs<D, T, C>(L, xs + (int64_t)f * L.Ns,
                                  (uint32_t)(rb0 + (int64_t)dy * L.Rp + (int64_t)dz * L.Pp), t, tn, v);
                static_for<0, M>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    static_for<0, 3>([&](auto xc) {
                        constexpr int dx = decltype(xc)::value - 1;
                        constexpr int o = off_index<D>(dx, dy, dz);
                        if constexpr (o >= 0) {
                            constexpr int w0 = sdiv_int<D>(0, o), w1 = sdiv_int<D>(1, o);
                            constexpr int w2 = D == 3 ? sdiv_int<D>(D - 1, o) : 0;
                            if constexpr (w0 != 0 || w1 != 0 || w2 != 0)
                                dv[q] += (C)(f == 0 ? w0 : (f == 1 ? w1 : w2)) * v[1 + q + dx];
                        }
                    });
                });
            }
        });
    }
    // pressure: C rows
    static_for<0, rhs_rows<D>()>([&](auto rc) {
        constexpr int dy = ROW_DY[decltype(rc)::value];
        constexpr int dz = D == 3 ? ROW_DZ[decltype(rc)::value] : 0;
        if constexpr (row_used<D, 2, 0>(dy, dz)) {
            C v[M + 2];
            row_runs<D, T, C>(L, xs + (int64_t)D * L.Ns, (uint32_t)(rb0 + (int64_t)dy * L.Rp + (int64_t)dz * L.Pp),
                              t, tn, v);
            static_for<0, M>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                static_for<0, 3>([&](auto xc) {
                    constexpr int dx = decltype(xc)::value - 1;
                    constexpr int o = off_index<D>(dx, dy, dz);
                    if constexpr (o >= 0) {
                        constexpr int w = sc_int<D>(o);
                        if constexpr (w != 0) cp[q] += (C)w * v[1 + q + dx];
                    }
                });
            });
        }
    });
    if (!act) return;
    const int m = L.n - 1;
    const C sdv = (C)(L.sB * (-kuhn_volume<D>() / (D + 1)));
    const C vol = (C)kuhn_volume<D>();
    constexpr int c0 = sc_int<D>(0);
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const int i = M * t + q;
        if (i < 1 || i > m) continue;
        const int64_t v = rb0 + (int64_t)q * L.q + t;
        const int ph = L.vphase_s[v];
        if (ph == SPECIAL) continue;
        const C sci = (C)L.sC * PrecU<C>::imu(L, ph);
        const C sv = sdv * dv[q] - sci * (vol * cp[q]) - (C)bs[(int64_t)D * L.Ns + v];
        if ((i + j + k) % M == 0) delta[v] = (T)(sv / (sci * (vol * (C)c0)));
        else sres[v] = (T)sv;
    }
}

// ----------------------------------------------------------------------------
// LDS-tiled z-marching passes of the levels above 65^3 (3D): the right-hand
// sides of the smoother and the operator applies.
//
// A workgroup owns a tile of ZT_X canonical x positions by ZT_Y rows and a
// chunk of zc planes of the interior.  One plane of every field its
// stencils read (the tile and a one-vertex ring around it) sits in LDS at a
// time, so every value comes from memory once per tile instead of once per
// stencil entry, with full-width loads; the loads of the next plane are
// issued before the current one is used and stored to the second slot
// after it.  Workgroup b runs on XCD b % 8; each XCD walks a slab of tile
// rows (x tiles fastest, then rows, then z chunks), so the tiles whose
// rings overlap share its L2.
constexpr int ZT_X = 64, ZT_Y = 4;
constexpr int ZT_W = ZT_X + 2, ZT_H = ZT_Y + 2, ZT_A = ZT_W * ZT_H;
constexpr int ZT_PER = (ZT_A + 255) / 256;   // loads per thread per field plane

struct ZTileGrid {
    int gx, gy, gys, gz, zc;   // tiles along x, y (per XCD slab), z chunks of zc planes
};

// The z chunk is as long as possible (each chunk reloads two ring planes)
// while the grid still offers about four workgroups per CU: 8 to 32 planes.
inline ZTileGrid ztile_grid(int n) {
    const int m = n - 1;
    ZTileGrid g;
    g.gx = (m + ZT_X - 1) / ZT_X;
    g.gy = (m + ZT_Y - 1) / ZT_Y;
    g.gys = (g.gy + NXCD - 1) / NXCD;
    const int per_layer = NXCD * g.gx * g.gys;
    const int want = std::max(1, (1024 + per_layer - 1) / per_layer);
    g.zc = std::min(32, std::max(8, (m + want - 1) / want));
    g.gz = (m + g.zc - 1) / g.zc;
    return g;
}

// tile origin (interior coordinates start at 1) and plane range of a
// workgroup; false for the padding workgroups of the last XCD slabs
__device__ __forceinline__ bool ztile_origin(const LevelView& L, ZTileGrid g, int& i0, int& j0, int& k0, int& k1) {
    const int bid = (int)blockIdx.x;
    const int xcd = bid & (NXCD - 1);
    const int idx = bid / NXCD;
    const int tx = idx % g.gx;
    const int r = idx / g.gx;
    const int ty = xcd * g.gys + r % g.gys;
    const int tz = r / g.gys;
    if (ty >= g.gy || tz >= g.gz) return false;
    i0 = 1 + tx * ZT_X;
    j0 = 1 + ty * ZT_Y;
    k0 = 1 + tz * g.zc;
    k1 = min(k0 + g.zc, L.n);      // planes k0 .. k1-1 (interior ends at n-1)
    return true;
}

// split-layout offset of (i, j, k) inside a field (3D, M = 4 colours)
__device__ __forceinline__ uint32_t sidx3(const LevelView& L, int i, int j, int k) {
    return (uint32_t)k * (uint32_t)L.Pp + (uint32_t)j * (uint32_t)L.Rp + (uint32_t)(i & 3) * (uint32_t)L.q +
           (uint32_t)(i >> 2);
}

// global loads of plane kk of NF fields (fields f0.. of the vector xs, in
// the colour-split layout if SPLIT, else canonical) for this thread's
// ZT_PER tile entries; entries past the lattice are 0
template <int NF, bool SPLIT, typename T, typename C>
__device__ __forceinline__ void ztile_fetch(const LevelView& L, const T* __restrict__ xs, int f0, int i0, int j0,
                                            int kk, C (&reg)[NF][ZT_PER]) {
    const int64_t fstride = SPLIT ? L.Ns : L.N;
#pragma unroll
    for (int q = 0; q < ZT_PER; ++q) {
        const int e = (int)threadIdx.x + 256 * q;
        const int r = e / ZT_W, c = e - r * ZT_W;
        const int ii = i0 - 1 + c, jj = j0 - 1 + r;
        const bool ok = e < ZT_A && ii <= L.n && jj <= L.n;
        const uint32_t off = !ok ? 0u
                             : SPLIT ? sidx3(L, ii, jj, kk)
                                     : (uint32_t)kk * (uint32_t)L.sz + (uint32_t)jj * (uint32_t)L.sy + (uint32_t)ii;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const C v = (C)ld32(xs + (int64_t)(f0 + f) * fstride, off);
            reg[f][q] = ok ? v : (C)0;
        }
    }
}

template <int NF, int NS, typename C>
__device__ __forceinline__ void ztile_store(C (*lds)[NS][ZT_A], int slot, const C (&reg)[NF][ZT_PER]) {
#pragma unroll
    for (int q = 0; q < ZT_PER; ++q) {
        const int e = (int)threadIdx.x + 256 * q;
        if (e < ZT_A) {
#pragma unroll
            for (int f = 0; f < NF; ++f) lds[f][slot][e] = reg[f][q];
        }
    }
}

// The streaming form of the z march, for passes whose rows are sums of
// weighted values: a thread reads only plane kk of the tile (its own
// position and the in-plane neighbours the stencil reaches) and adds each
// value into every row that reads it, row (i, j, kk - dz) for the offsets
// (dx, dy, dz) that land on it; the rows kk - 1, kk and kk + 1 are rolling
// sums in registers, and row kk - 1 is complete once plane kk is in.  Half
// the LDS reads of the three-plane ring, and two plane slots instead of
// three.  body(i, j, kk, slot of kk, emit): emit is set for active threads
// whose row kk - 1 lies in the chunk.
template <int NF, bool SPLIT, typename T, typename C, typename Body>
__device__ __forceinline__ void ztile_stream(const LevelView& L, ZTileGrid zg, const T* __restrict__ xs, int f0,
                                             C (*lds)[2][ZT_A], Body&& body) {
    int i0, j0, k0, k1;
    if (!ztile_origin(L, zg, i0, j0, k0, k1)) return;
    const int tx = (int)threadIdx.x & (ZT_X - 1), ty = (int)threadIdx.x / ZT_X;
    const int i = i0 + tx, j = j0 + ty;
    const bool active = i <= L.n - 1 && j <= L.n - 1;
    C reg[NF][ZT_PER];
    ztile_fetch<NF, SPLIT, T, C>(L, xs, f0, i0, j0, k0 - 1, reg);
    ztile_store<NF, 2, C>(lds, 0, reg);
    __syncthreads();
    int cur = 0;
    for (int kk = k0 - 1; kk <= k1; ++kk) {
        // the slot written here was last read before the previous barrier
        const bool pre = kk < k1;
        if (pre) ztile_fetch<NF, SPLIT, T, C>(L, xs, f0, i0, j0, kk + 1, reg);
        body(i, j, kk, cur, active && kk - 1 >= k0);
        if (pre) ztile_store<NF, 2, C>(lds, cur ^ 1, reg);
        __syncthreads();
        cur ^= 1;
    }
}

// s = B u - C p - g on interior isoviscous vertices, colour 0 finishing its
// first pressure Gauss-Seidel phase (delta = s / C_vv), as k_p_rhs_g.
// Streamed: dv[r], cp[r] hold the divergence and stabilisation sums of the
// rows kk - 1 (r = 0), kk (1) and kk + 1 (2).
template <typename T>
__global__ __launch_bounds__(256) void k_p_rhs_z(LevelView L, ZTileGrid zg, const T* __restrict__ xs,
                                                 const T* __restrict__ bs, T* __restrict__ sres, T* __restrict__ delta) {
    using C = typename Acc<T>::type;
    constexpr int D = 3;
    __shared__ C lds[D + 1][2][ZT_A];
    const C sdv = (C)(L.sB * (-kuhn_volume<D>() / (D + 1)));
    const C vol = (C)kuhn_volume<D>();
    constexpr int c0 = sc_int<D>(0);
    C dv[3] = {0, 0, 0}, cp[3] = {0, 0, 0};
    ztile_stream<D + 1, true, T, C>(L, zg, xs, 0, lds, [&](int i, int j, int kk, int slot, bool emit) {
        const int cen = (1 + (int)threadIdx.x / ZT_X) * ZT_W + 1 + ((int)threadIdx.x & (ZT_X - 1));
        static_for<0, KuhnTables<D>::NB>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            constexpr int dx = Kuhn<D>::T.off[o][0], dy = Kuhn<D>::T.off[o][1], dz = Kuhn<D>::T.off[o][2];
            constexpr int r = 1 - dz;          // the value at plane kk belongs to row kk - dz
            const int e = cen + dy * ZT_W + dx;
            static_for<0, D>([&](auto fc) {
                constexpr int f = decltype(fc)::value;
                constexpr int w = sdiv_int<D>(f, o);
                if constexpr (w != 0) dv[r] += (C)w * lds[f][slot][e];
            });
            constexpr int wc = sc_int<D>(o);
            if constexpr (wc != 0) cp[r] += (C)wc * lds[D][slot][e];
        });
        if (emit) {
            const int k = kk - 1;
            const uint32_t v = sidx3(L, i, j, k);
            const int ph = L.vphase_s[v];
            if (ph != SPECIAL) {
                const C sci = (C)L.sC * PrecU<C>::imu(L, ph);
                const C sv = sdv * dv[0] - sci * (vol * cp[0]) - (C)ld32(bs + (int64_t)D * L.Ns, v);
                if (((i + j + k) & 3) == 0) delta[v] = (T)(sv / (sci * (vol * (C)c0)));
                else sres[v] = (T)sv;
            }
        }
        dv[0] = dv[1]; dv[1] = dv[2]; dv[2] = 0;
        cp[0] = cp[1]; cp[1] = cp[2]; cp[2] = 0;
    });
}

// g = f - B^T p on interior isoviscous vertices, as k_vel_rhs_s; acc[r]
// holds the streamed sums of the rows kk - 1, kk and kk + 1.
template <typename T>
__global__ __launch_bounds__(256) void k_vel_rhs_z(LevelView L, ZTileGrid zg, const T* __restrict__ xs,
                                                   const T* __restrict__ bs, T* __restrict__ g) {
    using C = typename Acc<T>::type;
    constexpr int D = 3;
    __shared__ C lds[1][2][ZT_A];
    const C sbv = (C)(L.sB * (-kuhn_volume<D>() / (D + 1)));
    C acc[3][D] = {};
    ztile_stream<1, true, T, C>(L, zg, xs, D, lds, [&](int i, int j, int kk, int slot, bool emit) {
        const int cen = (1 + (int)threadIdx.x / ZT_X) * ZT_W + 1 + ((int)threadIdx.x & (ZT_X - 1));
        static_for<0, KuhnTables<D>::NB>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            constexpr int dx = Kuhn<D>::T.off[o][0], dy = Kuhn<D>::T.off[o][1], dz = Kuhn<D>::T.off[o][2];
            constexpr int r = 1 - dz;          // the value at plane kk belongs to row kk - dz
            constexpr bool used = sbt_int<D>(0, o) != 0 || sbt_int<D>(1, o) != 0 || sbt_int<D>(2, o) != 0;
            if constexpr (used) {
                const C pv = lds[0][slot][cen + dy * ZT_W + dx];
                static_for<0, D>([&](auto lc) {
                    constexpr int l = decltype(lc)::value;
                    constexpr int w = sbt_int<D>(l, o);
                    if constexpr (w != 0) acc[r][l] += (C)w * pv;
                });
            }
        });
        if (emit) {
            const uint32_t v = sidx3(L, i, j, kk - 1);
            if (L.vphase_s[v] != SPECIAL) {
#pragma unroll
                for (int l = 0; l < D; ++l)
                    g[(int64_t)l * L.Ns + v] = (T)((C)ld32(bs + (int64_t)l * L.Ns, v) - sbv * acc[0][l]);
            }
        }
#pragma unroll
        for (int l = 0; l < D; ++l) {
            acc[0][l] = acc[1][l]; acc[1][l] = acc[2][l]; acc[2][l] = 0;
        }
    });
}

// Operator apply / residual on the interior isoviscous vertices of a large
// 3D level (canonical layout), as apply_bulk_body: the streamed LDS z march
// with the compile-time integer stencils of the Kuhn lattice (viscous block times
// |T|, B and B^T times -|T|/(d+1), C times |T|).
template <int F, int BLK, int MODE, typename T>
__global__ __launch_bounds__(256) void k_apply_z(LevelView L, ZTileGrid zg, const T* __restrict__ x,
                                                 const T* __restrict__ b, T* __restrict__ y) {
    using C = typename Acc<T>::type;
    constexpr int D = 3;
    constexpr int NF = (BLK == BLOCK_FULL) ? D + 1 : D;
    __shared__ C lds[NF][2][ZT_A];
    const C vol = (C)kuhn_volume<D>();
    const C bvol = (C)(-kuhn_volume<D>() / (D + 1));
    // streamed sums of the rows kk - 1 (index 0), kk (1) and kk + 1 (2)
    C av[3][D] = {}, bt[3][D] = {}, dv[3] = {0, 0, 0}, cp[3] = {0, 0, 0};
    ztile_stream<NF, false, T, C>(L, zg, x, 0, lds, [&](int i, int j, int kk, int slot, bool emit) {
        const int cen = (1 + (int)threadIdx.x / ZT_X) * ZT_W + 1 + ((int)threadIdx.x & (ZT_X - 1));
        static_for<0, KuhnTables<D>::NB>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            constexpr int dx = Kuhn<D>::T.off[o][0], dy = Kuhn<D>::T.off[o][1], dz = Kuhn<D>::T.off[o][2];
            constexpr int r = 1 - dz;          // the value at plane kk belongs to row kk - dz
            const int e = cen + dy * ZT_W + dx;
            static_for<0, D>([&](auto kc) {
                constexpr int kf = decltype(kc)::value;
                constexpr bool used = svis_int<D>(F, 0, kf, o) != 0 || svis_int<D>(F, 1, kf, o) != 0 ||
                                      svis_int<D>(F, 2, kf, o) != 0 || (BLK == BLOCK_FULL && sdiv_int<D>(kf, o) != 0);
                if constexpr (used) {
                    const C u = lds[kf][slot][e];
                    static_for<0, D>([&](auto lc) {
                        constexpr int l = decltype(lc)::value;
                        constexpr int wv = svis_int<D>(F, l, kf, o);
                        if constexpr (wv != 0) av[r][l] += (C)wv * u;
                    });
                    if constexpr (BLK == BLOCK_FULL) {
                        constexpr int wd = sdiv_int<D>(kf, o);
                        if constexpr (wd != 0) dv[r] += (C)wd * u;
                    }
                }
            });
            if constexpr (BLK == BLOCK_FULL) {
                constexpr bool pused = sbt_int<D>(0, o) != 0 || sbt_int<D>(1, o) != 0 || sbt_int<D>(2, o) != 0 ||
                                       sc_int<D>(o) != 0;
                if constexpr (pused) {
                    const C pv = lds[D][slot][e];
                    static_for<0, D>([&](auto lc) {
                        constexpr int l = decltype(lc)::value;
                        constexpr int wb = sbt_int<D>(l, o);
                        if constexpr (wb != 0) bt[r][l] += (C)wb * pv;
                    });
                    constexpr int wc = sc_int<D>(o);
                    if constexpr (wc != 0) cp[r] += (C)wc * pv;
                }
            }
        });
        if (emit) {
            const int k = kk - 1;
            const int64_t v = (int64_t)i + (int64_t)j * L.sy + (int64_t)k * L.sz;
            const int ph = L.vphase[v];
            if (ph != SPECIAL) {
                const C smu = PrecU<C>::mu(L, ph) * (C)L.sA * vol;
                const C sb = (C)L.sB * bvol;
                C out[D + 1];
#pragma unroll
                for (int l = 0; l < D; ++l) out[l] = smu * av[0][l] + (BLK == BLOCK_FULL ? sb * bt[0][l] : (C)0);
                out[D] = (BLK == BLOCK_FULL) ? sb * dv[0] - (C)L.sC * PrecU<C>::imu(L, ph) * (vol * cp[0]) : (C)0;
#pragma unroll
                for (int f = 0; f <= D; ++f) {
                    const int64_t ef = (int64_t)f * L.N + v;
                    if (MODE == MODE_RESID)
                        y[ef] = (BLK == BLOCK_FULL || f < D) ? (T)((C)b[ef] - out[f]) : (T)0.0f;
                    else
                        y[ef] = (T)out[f];
                }
            }
        }
#pragma unroll
        for (int l = 0; l < D; ++l) {
            av[0][l] = av[1][l]; av[1][l] = av[2][l]; av[2][l] = 0;
            bt[0][l] = bt[1][l]; bt[1][l] = bt[2][l]; bt[2][l] = 0;
        }
        dv[0] = dv[1]; dv[1] = dv[2]; dv[2] = 0;
        cp[0] = cp[1]; cp[1] = cp[2]; cp[2] = 0;
    });
}

template <int D, int F, bool BWD, typename T>
__device__ __forceinline__ void gs_vel_body(const LevelView& L, int colour, int64_t bid, int tid,
                                            T* __restrict__ xs, const T* __restrict__ g) {
    using C = typename Acc<T>::type;
    constexpr int NB = KuhnTables<D>::NB;
    int s;
    int64_t v;
    if (!split_colour_vertex<D>(L, colour, bid, tid, s, v)) return;
    const XOff xo = x_offsets<D>(L, s);
    const auto& E = ETab<D, C>::get();
    // every load is issued before the phase test (all addresses are
    // interior, so the loads are in bounds for special vertices too)
    const int ph = L.vphase_s[v];
    C gl[D];
#pragma unroll
    for (int l = 0; l < D; ++l) gl[l] = (C)g[(int64_t)l * L.Ns + v];
    if (F == FORM_STRAIN) {
        C U[D][NB];
        load_split<D, D, T, C>(L, xs, v, xo, 0, U);
        if (ph == SPECIAL) return;
        const C smu = PrecU<C>::mu(L, ph) * (C)L.sA;
        C r[D], Dm[D][D], du[D];
#pragma unroll
        for (int l = 0; l < D; ++l) {
            C acc = 0;
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
#pragma unroll
                for (int o = 0; o < NB; ++o) acc += E.Svis[1][l][kk][o] * U[kk][o];
                Dm[l][kk] = smu * E.Svis[1][l][kk][0];
            }
            r[l] = gl[l] - smu * acc;
        }
        block_gs_update<D, F, BWD, C>(r, Dm, du);
#pragma unroll
        for (int l = 0; l < D; ++l) xs[(int64_t)l * L.Ns + v] = (T)(U[l][0] + du[l]);
    } else {
        // decoupled components: u_l = (g_l - mu sA sum_nb w u_l) / (mu sA w_0);
        // the neighbours are the runs of colours c - 1 and c + 1 only
        C nb[D][2 * D];
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
            for (int o = 1; o <= 2 * D; ++o) nb[l][o - 1] = (C)xs[(int64_t)l * L.Ns + v + snb<D>(L, xo, o)];
        if (ph == SPECIAL) return;
        const C smu = PrecU<C>::mu(L, ph) * (C)L.sA;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            C acc = 0;
#pragma unroll
            for (int o = 1; o <= 2 * D; ++o) acc += E.Svis[0][l][l][o] * nb[l][o - 1];
            const C w0 = smu * E.Svis[0][l][l][0];
            xs[(int64_t)l * L.Ns + v] = (T)((gl[l] - smu * acc) / w0);
        }
    }
}

template <int D, int F, bool BWD, typename T>
__device__ __forceinline__ void gs_vel_special_body(const LevelView& L, int colour, int64_t rel,
                                                    T* __restrict__ xs, const T* __restrict__ bs) {
    using C = typename Acc<T>::type;
    constexpr int NB = KuhnTables<D>::NB;
    const int64_t sp = L.spec_off[colour] + rel;
    if (sp >= L.spec_off[colour + 1]) return;
    int ijk[3];
    vertex_ijk<D>(L, L.spec[sp], ijk);
    const bool bnd = on_boundary<D>(L, ijk);
    if (bnd && !L.freeslip) return;              // no-slip: every component fixed
    const int64_t v = sidx<D>(L, ijk[0], ijk[1], ijk[2]);
    C U[D][NB], P[1][NB];
    load_guarded_split<D, D, T, C>(L, xs, ijk, 0, U);
    load_guarded_split<D, 1, T, C>(L, xs, ijk, D, P);
    RowAcc<D, F, true, false, C> r;
    element_rows<D, F, true, false, true, false, C>(L, sp, U, P[0], P[0], r);
    C res[D], Dm[D][D], du[D];
#pragma unroll
    for (int l = 0; l < D; ++l) {
        res[l] = (C)bs[(int64_t)l * L.Ns + v] - (C)L.sB * r.abt[l] - (C)L.sA * r.au[l];
#pragma unroll
        for (int k = 0; k < D; ++k) Dm[l][k] = (C)L.sA * r.Dm[l][k];
    }
    if (bnd) {
        // free-slip: a fixed (normal) component keeps its zero; its row and
        // column leave the point block
#pragma unroll
        for (int l = 0; l < D; ++l) {
            if (!vel_fixed<D>(L, ijk, l)) continue;
            res[l] = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) { Dm[l][k] = 0; Dm[k][l] = 0; }
            Dm[l][l] = 1;
        }
    }
    block_gs_update<D, F, BWD, C>(res, Dm, du);
#pragma unroll
    for (int l = 0; l < D; ++l) xs[(int64_t)l * L.Ns + v] = (T)(U[l][0] + du[l]);
}

// Pressure: s = B u - C p - g on interior isoviscous vertices (u and p are
// fixed during the pressure sweep), then one forward colour sweep of
// Gauss-Seidel on C delta = s from delta = 0.  This form (one vertex per
// thread, merged with the colour-0 special rows) serves the levels up to
// 65^3; k_p_rhs_g below serves the larger ones.
//
// The first colour phase of the sweep is folded into this pass: every
// neighbour of a colour-0 vertex has another colour and still holds
// delta = 0, so its update is s / (C_vv) and s need not be stored.  The
// special rows of colour 0 (element loops, their own s) read only
// neighbours of other colours and write only their own delta, so they run
// in the same grid: one-wave workgroups, four per 256-thread bulk group,
// special rows from workgroup 4 nbulk on.  (On larger levels they have their
// own launch, which keeps the s pass at half the registers of the element
// loop.)
template <int D, typename T>
__device__ __forceinline__ void gs_p_special_body(const LevelView& L, int colour, int64_t rel,
                                                  const T* __restrict__ xs, const T* __restrict__ bs,
                                                  T* __restrict__ delta);

template <int D, typename T>
__global__ __launch_bounds__(64) void k_p_rhs_s(LevelView L, const T* __restrict__ xs, const T* __restrict__ bs,
                                                T* __restrict__ sres, T* __restrict__ delta, int64_t nbulk) {
    using C = typename Acc<T>::type;
    constexpr int NB = KuhnTables<D>::NB;
    int64_t bid = blockIdx.x;
    int tid = threadIdx.x;
    if (bid >= 4 * nbulk) {
        gs_p_special_body<D, T>(L, 0, (bid - 4 * nbulk) * 64 + tid, xs, bs, delta);
        return;
    }
    tid += (int)(bid & 3) * 64;
    bid >>= 2;
    int s, colour;
    int64_t v;
    if (!split_all_vertex<D>(L, bid, tid, s, v, colour)) return;
    const XOff xo = x_offsets<D>(L, s);
    const auto& E = ETab<D, C>::get();
    const int ph = L.vphase_s[v];
    C U[D][NB], P[1][NB];
    load_split<D, D, T, C>(L, xs, v, xo, 0, U);
    load_split<D, 1, T, C>(L, xs, v, xo, D, P);
    const C bp = (C)bs[(int64_t)D * L.Ns + v];
    if (ph == SPECIAL) return;
    C dv = 0;
#pragma unroll
    for (int kk = 0; kk < D; ++kk)
#pragma unroll
        for (int o = 1; o < NB; ++o) dv += E.Sdiv[kk][o] * U[kk][o];
    C cp = E.Sc[0] * P[0][0];
#pragma unroll
    for (int o = 1; o <= 2 * D; ++o) cp += E.Sc[o] * P[0][o];
    const C sci = (C)L.sC * PrecU<C>::imu(L, ph);
    const C sv = (C)L.sB * dv - sci * cp - bp;
    if (colour == 0) delta[v] = (T)(sv / (sci * E.Sc[0]));
    else sres[v] = (T)sv;
}

template <int D, typename T>
__device__ __forceinline__ void gs_p_body(const LevelView& L, int colour, int64_t bid, int tid,
                                          const T* __restrict__ sres, T* __restrict__ delta) {
    using C = typename Acc<T>::type;
    int s;
    int64_t v;
    if (!split_colour_vertex<D>(L, colour, bid, tid, s, v)) return;
    const XOff xo = x_offsets<D>(L, s);
    const auto& E = ETab<D, C>::get();
    const int ph = L.vphase_s[v];
    C nb[2 * D];
#pragma unroll
    for (int o = 1; o <= 2 * D; ++o) nb[o - 1] = (C)delta[v + snb<D>(L, xo, o)];
    const C sv = (C)sres[v];
    if (ph == SPECIAL) return;
    C cd = 0;
#pragma unroll
    for (int o = 1; o <= 2 * D; ++o) cd += E.Sc[o] * nb[o - 1];
    const C sci = (C)L.sC * PrecU<C>::imu(L, ph);
    delta[v] = (T)((sv - sci * cd) / (sci * E.Sc[0]));
}

template <int D, typename T>
__device__ __forceinline__ void gs_p_special_body(const LevelView& L, int colour, int64_t rel,
                                                  const T* __restrict__ xs, const T* __restrict__ bs,
                                                  T* __restrict__ delta) {
    using C = typename Acc<T>::type;
    constexpr int NB = KuhnTables<D>::NB;
    const int64_t sp = L.spec_off[colour] + rel;
    if (sp >= L.spec_off[colour + 1]) return;
    int ijk[3];
    vertex_ijk<D>(L, L.spec[sp], ijk);
    const int64_t v = sidx<D>(L, ijk[0], ijk[1], ijk[2]);
    C U[D][NB], P[1][NB], Dl[1][NB];
    load_guarded_split<D, D, T, C>(L, xs, ijk, 0, U);
    load_guarded_split<D, 1, T, C>(L, xs, ijk, D, P);
    load_guarded_split<D, 1, T, C>(L, delta, ijk, 0, Dl);
    RowAcc<D, FORM_GRADIENT, false, true, C> r;
    element_rows<D, FORM_GRADIENT, false, true, true, true, C>(L, sp, U, P[0], Dl[0], r);
    const C sres = (C)L.sB * r.bdiv - (C)L.sC * r.cp - (C)bs[(int64_t)D * L.Ns + v];
    delta[v] = (T)((sres - (C)L.sC * r.cd) / ((C)L.sC * r.cjj));
}

// One colour phase, three launch shapes: bulk only, special only, and both
// in one grid for small levels, where the launch latency of two kernels
// costs more than the lower occupancy of the merged one.  The merged grid is
// made of one-wave workgroups: four per 256-thread bulk group first, then
// the special rows.
// The velocity special-only kernel uses one-wave workgroups, so the
// scattered interface rows spread over every CU; under no-slip it starts at
// the first interior row of the colour (the boundary rows before it are
// fixed).  In the pressure kernel every row does work; long lists keep
// 4-wave groups (neighbouring boundary rows share a CU's L1), short ones use
// one wave per group to reach more CUs.  The special-only kernels hand the
// XCDs runs of consecutive blocks of their list (xcd_group_remap).
constexpr int SPEC_WG = 64;
template <int D, int F, bool BWD, typename T>
__global__ __launch_bounds__(256) void k_gs_vel_s(LevelView L, int colour, T* __restrict__ xs,
                                                  const T* __restrict__ g) {
    gs_vel_body<D, F, BWD, T>(L, colour, blockIdx.x, threadIdx.x, xs, g);
}

template <int D, int F, bool BWD, typename T>
__global__ __launch_bounds__(SPEC_WG) void k_gs_vel_special_s(LevelView L, int colour, T* __restrict__ xs,
                                                              const T* __restrict__ bs) {
    const int64_t skip = L.freeslip ? 0 : L.spec_mid[colour] - L.spec_off[colour];
    gs_vel_special_body<D, F, BWD, T>(L, colour, skip + xcd_group_remap(blockIdx.x, gridDim.x) * SPEC_WG + threadIdx.x,
                                      xs, bs);
}

template <int D, int F, bool BWD, typename T>
__global__ __launch_bounds__(64) void k_gs_vel_m(LevelView L, int colour, T* __restrict__ xs,
                                                 const T* __restrict__ g, const T* __restrict__ bs,
                                                 int64_t nbulk) {
    const int64_t b = blockIdx.x;
    if (b < 4 * nbulk) gs_vel_body<D, F, BWD, T>(L, colour, b >> 2, (int)(b & 3) * 64 + threadIdx.x, xs, g);
    else gs_vel_special_body<D, F, BWD, T>(L, colour, (b - 4 * nbulk) * 64 + threadIdx.x, xs, bs);
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_gs_p_s(LevelView L, int colour, const T* __restrict__ sres,
                                                T* __restrict__ delta) {
    gs_p_body<D, T>(L, colour, blockIdx.x, threadIdx.x, sres, delta);
}

template <int D, typename T, int WG>
__global__ __launch_bounds__(WG) void k_gs_p_special_s(LevelView L, int colour, const T* __restrict__ xs,
                                                       const T* __restrict__ bs, T* __restrict__ delta) {
    gs_p_special_body<D, T>(L, colour, xcd_group_remap(blockIdx.x, gridDim.x) * WG + threadIdx.x, xs, bs, delta);
}

template <int D, typename T>
__global__ __launch_bounds__(64) void k_gs_p_m(LevelView L, int colour, const T* __restrict__ sres,
                                               const T* __restrict__ xs, const T* __restrict__ bs,
                                               T* __restrict__ delta, int64_t nbulk) {
    const int64_t b = blockIdx.x;
    if (b < 4 * nbulk) gs_p_body<D, T>(L, colour, b >> 2, (int)(b & 3) * 64 + threadIdx.x, sres, delta);
    else gs_p_special_body<D, T>(L, colour, (b - 4 * nbulk) * 64 + threadIdx.x, xs, bs, delta);
}

// p += w d, then d = 0: the pressure correction of a smoothing step is
// applied and its buffer left cleared for the next step's sweep
template <typename T>
__global__ void k_axpy_clear(T* __restrict__ p, T* __restrict__ d, typename Acc<T>::type w, int64_t n) {
    using C = typename Acc<T>::type;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        p[e] = (T)((C)p[e] + w * (C)d[e]);
        d[e] = (T)(C)0;
    }
}

template <typename T>
__global__ void k_fill_t(T* __restrict__ x, int64_t n, typename Acc<T>::type val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) x[e] = val;
}

// ----------------------------------------------------------------------------
// transfers: P1 interpolation between nested Kuhn lattices.  A fine vertex
// with even coordinates is a coarse vertex; otherwise it is the midpoint
// of the coarse edge along its odd-coordinate pattern (a Kuhn direction).

template <int D, typename T>
__global__ __launch_bounds__(256) void k_restrict_t(LevelView Lf, LevelView Lc,
                                                    const T* __restrict__ rf,
                                                    T* __restrict__ rc) {
    using C = typename Acc<T>::type;
    constexpr auto& TT = Kuhn<D>::T;
    constexpr int NB = KuhnTables<D>::NB;
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= Lc.N) return;
    int c[3];
    vertex_ijk<D>(Lc, I, c);
    const int64_t F = 2 * c[0] + 2 * c[1] * Lf.sy + 2 * c[2] * Lf.sz;
    C acc[D + 1];
#pragma unroll
    for (int f = 0; f <= D; ++f) acc[f] = (C)rf[(int64_t)f * Lf.N + F];
#pragma unroll
    for (int o = 1; o < NB; ++o) {
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int q = 2 * c[a] + TT.off[o][a];
            in = in && q >= 0 && q <= Lf.n;
        }
        if (!in) continue;
        const int64_t fo = F + nb_lin<D>(Lf, o);
#pragma unroll
        for (int f = 0; f <= D; ++f) acc[f] += (C)0.5 * (C)rf[(int64_t)f * Lf.N + fo];
    }
#pragma unroll
    for (int f = 0; f <= D; ++f)
        rc[(int64_t)f * Lc.N + I] = (f < D && vel_fixed<D>(Lc, c, f < D ? f : 0)) ? (T)0.0f : (T)acc[f];
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_prolong_t(LevelView Lf, LevelView Lc,
                                                   const T* __restrict__ ec,
                                                   T* __restrict__ xf) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Lf.N) return;
    int a[3];
    vertex_ijk<D>(Lf, v, a);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    bool odd = false;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const int o = a[q] & 1;
        odd = odd || o;
        lo[q] = (a[q] - o) >> 1;
        hi[q] = (a[q] + o) >> 1;
    }
    const int64_t cl = lo[0] + lo[1] * Lc.sy + lo[2] * Lc.sz;
    const int64_t ch = hi[0] + hi[1] * Lc.sy + hi[2] * Lc.sz;
#pragma unroll
    for (int f = 0; f <= D; ++f) {
        const T* e = ec + (int64_t)f * Lc.N;
        using C = typename Acc<T>::type;
        const C val = odd ? (C)0.5 * ((C)e[cl] + (C)e[ch]) : (C)e[cl];
        T* dst = xf + (int64_t)f * Lf.N + v;
        *dst = (T)((C)*dst + val);
    }
}

// ----------------------------------------------------------------------------
// reductions (two-stage, deterministic)

constexpr int RED_BLOCKS = 1024;

template <int B>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < B / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

template <typename T, bool SQUARE = true>
__global__ __launch_bounds__(256) void k_sumsq_partial(const T* __restrict__ x, int64_t N,
                                                       int nf, double* __restrict__ partial) {
    __shared__ double sh[4];
    for (int f = 0; f < nf; ++f) {
        double acc = 0;
        const T* xf = x + (int64_t)f * N;
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
            const double t = (double)(typename Acc<T>::type)xf[e];
            acc += SQUARE ? t * t : t;
        }
        const double s = block_sum<256>(acc, sh);
        if (threadIdx.x == 0) partial[(int64_t)f * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int nblk,
                                                   int nf, double* __restrict__ out) {
    __shared__ double sh[4];
    for (int f = 0; f < nf; ++f) {
        double acc = 0;
        for (int e = threadIdx.x; e < nblk; e += 256) acc += partial[(int64_t)f * nblk + e];
        const double s = block_sum<256>(acc, sh);
        if (threadIdx.x == 0) out[f] = s;
    }
}

// multi-dot: partial[i * gridDim.x + blk] = sum over the block's elements of
// V_i w, 16 vectors per workgroup row (blockIdx.y) so w is read once per
// 16 dot products; vector k (i == k) is w itself when with_self is set.
constexpr int MD_TILE = 16;
constexpr int KRY_UNROLL = 8;   // basis vectors read per step of the combination kernels
__global__ __launch_bounds__(256) void k_multidot_partial(const double* __restrict__ V, int64_t ldv,
                                                          int k, const double* __restrict__ w,
                                                          int64_t n, double* __restrict__ partial,
                                                          int with_self) {
    __shared__ double sh[MD_TILE][4];
    const int i0 = blockIdx.x * MD_TILE;          // tile fastest: w is re-read from L2
    const int nblk = gridDim.y, bid = blockIdx.y;
    const int kk = k + with_self;
    const int cnt = min(MD_TILE, kk - i0);
    double acc[MD_TILE];
#pragma unroll
    for (int q = 0; q < MD_TILE; ++q) acc[q] = 0;
    // rows past the tile's end re-read its last row (a cache hit) and are
    // dropped by the select, so every load of an element is issued before
    // the first wait
    const double* rows[MD_TILE];
#pragma unroll
    for (int q = 0; q < MD_TILE; ++q) {
        const int i = i0 + min(q, cnt - 1);
        rows[q] = (i < k) ? V + (int64_t)i * ldv : w;
    }
    for (int64_t e = (int64_t)bid * 256 + threadIdx.x; e < n; e += (int64_t)nblk * 256) {
        const double we = w[e];
        double vi[MD_TILE];
#pragma unroll
        for (int q = 0; q < MD_TILE; ++q) vi[q] = rows[q][e];
#pragma unroll
        for (int q = 0; q < MD_TILE; ++q) acc[q] += (q < cnt) ? vi[q] * we : 0.0;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < MD_TILE; ++q) {
        double v = acc[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) sh[q][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        const int q = threadIdx.x;
        partial[(int64_t)(i0 + q) * nblk + bid] = sh[q][0] + sh[q][1] + sh[q][2] + sh[q][3];
    }
}

// EPT consecutive doubles per lane: EPT == 2 reads them with one 16-byte
// load (the caller guarantees even n, even leading dimensions and 16-byte
// aligned vectors)
template <int EPT>
__device__ __forceinline__ void ld_ept(const double* __restrict__ p, double (&o)[EPT]) {
    if constexpr (EPT == 2) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 t = *reinterpret_cast<const d2*>(p);
        o[0] = t.x;
        o[1] = t.y;
    } else {
        o[0] = p[0];
    }
}
template <int EPT>
__device__ __forceinline__ void st_ept(double* __restrict__ p, const double (&o)[EPT]) {
    if constexpr (EPT == 2) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        d2 t;
        t.x = o[0];
        t.y = o[1];
        *reinterpret_cast<d2*>(p) = t;
    } else {
        p[0] = o[0];
    }
}

// One element range of the dot pass for a tile of basis rows; FULL tiles
// (cnt == MD_TILE) accumulate without the row mask.  All row loads of an
// element are issued before the first wait.
template <int EPT, bool FULL>
__device__ __forceinline__ void dots2_range(const double* const (&rows)[MD_TILE], int cnt,
                                            const double* __restrict__ a, const double* __restrict__ b,
                                            int64_t n, int64_t e0, int64_t stride, bool extras,
                                            double (&acc_a)[MD_TILE], double (&acc_b)[MD_TILE],
                                            double (&ex)[3]) {
    for (int64_t e = e0; e < n; e += stride) {
        double ae[EPT], be[EPT], vi[MD_TILE][EPT];
        ld_ept<EPT>(a + e, ae);
        ld_ept<EPT>(b + e, be);
#pragma unroll
        for (int q = 0; q < MD_TILE; ++q) ld_ept<EPT>(rows[q] + e, vi[q]);
#pragma unroll
        for (int q = 0; q < MD_TILE; ++q) {
            double sa = 0, sb = 0;
#pragma unroll
            for (int u = 0; u < EPT; ++u) { sa += vi[q][u] * ae[u]; sb += vi[q][u] * be[u]; }
            if (FULL || q < cnt) { acc_a[q] += sa; acc_b[q] += sb; }
        }
        if (extras) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) { ex[0] += ae[u] * ae[u]; ex[1] += ae[u] * be[u]; ex[2] += be[u] * be[u]; }
        }
    }
}

// Gram-Schmidt with delayed reorthogonalisation: one pass computes, for a
// tile of basis vectors V_i, the dot products V_i.a and V_i.b; tile 0 also
// accumulates a.a, a.b and b.b.  Partial sums per block; slots [0, k) hold
// V.a, [k, 2k) V.b, then a.a, a.b, b.b.
template <int EPT>
__global__ __launch_bounds__(256) void k_dots2_partial(const double* __restrict__ V, int64_t ldv, int k,
                                                       const double* __restrict__ a,
                                                       const double* __restrict__ b, int64_t n,
                                                       double* __restrict__ partial) {
    constexpr int NX = 3;
    // the vector tile is the fastest block index, so the tiles that share an
    // element range run together and re-read a and b from L2
    __shared__ double sh[2 * MD_TILE + NX][4];
    const int i0 = blockIdx.x * MD_TILE;
    const int nblk = gridDim.y, bid = blockIdx.y;
    const int cnt = max(0, min(MD_TILE, k - i0));
    const bool extras = blockIdx.x == 0;
    double acc_a[MD_TILE], acc_b[MD_TILE], ex[NX] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < MD_TILE; ++q) { acc_a[q] = 0; acc_b[q] = 0; }
    // rows past the tile's end re-read its last row (a cache hit) and are
    // masked; k == 0 reads a in place of a row
    const double* rows[MD_TILE];
#pragma unroll
    for (int q = 0; q < MD_TILE; ++q)
        rows[q] = cnt > 0 ? V + (int64_t)(i0 + min(q, cnt - 1)) * ldv : a;
    const int64_t e0 = ((int64_t)bid * 256 + threadIdx.x) * EPT, stride = (int64_t)nblk * 256 * EPT;
    if (cnt == MD_TILE) dots2_range<EPT, true>(rows, cnt, a, b, n, e0, stride, extras, acc_a, acc_b, ex);
    else dots2_range<EPT, false>(rows, cnt, a, b, n, e0, stride, extras, acc_a, acc_b, ex);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 2 * MD_TILE + NX; ++q) {
        double v = q < MD_TILE ? acc_a[q] : (q < 2 * MD_TILE ? acc_b[q - MD_TILE] : ex[q - 2 * MD_TILE]);
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) sh[q][wid] = v;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const double tot = (t < 2 * MD_TILE + NX) ? sh[t][0] + sh[t][1] + sh[t][2] + sh[t][3] : 0.0;
    if (t < cnt) partial[(int64_t)(i0 + t) * nblk + bid] = tot;
    else if (t >= MD_TILE && t < MD_TILE + cnt)
        partial[(int64_t)(k + i0 + t - MD_TILE) * nblk + bid] = tot;
    else if (extras && t >= 2 * MD_TILE && t < 2 * MD_TILE + NX)
        partial[(int64_t)(2 * k + t - 2 * MD_TILE) * nblk + bid] = tot;
}

// out[f] = sum of the nblk partials of slot f (one block per slot)
__global__ __launch_bounds__(256) void k_sum_slots(const double* __restrict__ partial, int nblk,
                                                   double* __restrict__ out) {
    __shared__ double sh[4];
    const int f = blockIdx.x;
    double acc = 0;
    for (int e = threadIdx.x; e < nblk; e += 256) acc += partial[(int64_t)f * nblk + e];
    const double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) out[f] = s;
}

// Second pass of the delayed scheme: with c = V^T u and d = V^T w over the
// k finished basis vectors (u = column k of V, the previous projected
// vector), finish column k as v = (u - V c) / alpha and store the new
// projected vector (w - V d - e v) / s in column k + 1.  EPT elements per
// lane; KRY_UNROLL rows in flight; the sums keep the order i = 0..k-1.
template <int EPT>
__global__ __launch_bounds__(256) void k_dcgs_update_t(double* __restrict__ V, int64_t ldv, int k,
                                                       const double* __restrict__ c,
                                                       const double* __restrict__ d,
                                                       const double* __restrict__ w, double inv_alpha,
                                                       double ecoef, double inv_s, int64_t n) {
    const int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * EPT;
    if (e >= n) return;
    double s1[EPT], s2[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) { s1[u] = 0; s2[u] = 0; }
    int i = 0;
    for (; i + KRY_UNROLL <= k; i += KRY_UNROLL) {
        double vi[KRY_UNROLL][EPT];
#pragma unroll
        for (int r = 0; r < KRY_UNROLL; ++r) ld_ept<EPT>(V + (int64_t)(i + r) * ldv + e, vi[r]);
#pragma unroll
        for (int r = 0; r < KRY_UNROLL; ++r) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) { s1[u] += c[i + r] * vi[r][u]; s2[u] += d[i + r] * vi[r][u]; }
        }
    }
    for (; i < k; ++i) {
        double vi[EPT];
        ld_ept<EPT>(V + (int64_t)i * ldv + e, vi);
#pragma unroll
        for (int u = 0; u < EPT; ++u) { s1[u] += c[i] * vi[u]; s2[u] += d[i] * vi[u]; }
    }
    double uk[EPT], we[EPT], v[EPT], nx[EPT];
    ld_ept<EPT>(V + (int64_t)k * ldv + e, uk);
    ld_ept<EPT>(w + e, we);
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        v[u] = (uk[u] - s1[u]) * inv_alpha;
        nx[u] = (we[u] - s2[u] - ecoef * v[u]) * inv_s;
    }
    st_ept<EPT>(V + (int64_t)k * ldv + e, v);
    st_ept<EPT>(V + (int64_t)(k + 1) * ldv + e, nx);
}

__global__ __launch_bounds__(256) void k_multiaxpy_t(double* __restrict__ y, const double* __restrict__ X,
                                                     int64_t ldx, int k, const double* __restrict__ c,
                                                     double alpha, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    double acc = 0;
    int i = 0;
    for (; i + KRY_UNROLL <= k; i += KRY_UNROLL) {
        double xi[KRY_UNROLL];
#pragma unroll
        for (int u = 0; u < KRY_UNROLL; ++u) xi[u] = X[(int64_t)(i + u) * ldx + e];
#pragma unroll
        for (int u = 0; u < KRY_UNROLL; ++u) acc += c[i + u] * xi[u];
    }
    for (; i < k; ++i) acc += c[i] * X[(int64_t)i * ldx + e];
    y[e] += alpha * acc;
}

__global__ __launch_bounds__(256) void k_scale_t(double* __restrict__ y, double a,
                                                 const double* __restrict__ x, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) y[e] = a * x[e];
}

__global__ __launch_bounds__(256) void k_axpby_t(double* __restrict__ y, double a,
                                                 const double* __restrict__ x, double b, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) y[e] = a * x[e] + b * y[e];
}

template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_convert_t(const Ti* __restrict__ in, To* __restrict__ out,
                                                   int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) out[e] = (To)(typename Acc<To>::type)(typename Acc<Ti>::type)in[e];
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_t(const T* __restrict__ x, const int32_t* __restrict__ idx,
                                                  int64_t m, double* __restrict__ out, FieldMul fm) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m) return;
    const int64_t i = idx[e];
    const double v = (double)(typename Acc<T>::type)x[i];
    out[e] = fm.on ? v * fm.m[i / fm.N] : v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_t(const double* __restrict__ in,
                                                   const int32_t* __restrict__ idx, int64_t m,
                                                   T* __restrict__ x, FieldMul fm) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m) return;
    const int64_t i = idx[e];
    x[i] = (T)(typename Acc<T>::type)(fm.on ? in[e] * fm.m[i / fm.N] : in[e]);
}

template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_scale_convert_t(const Ti* __restrict__ in, To* __restrict__ out,
                                                         int64_t N, const double* __restrict__ mul) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N) return;
    const int f = blockIdx.y;
    const double v = (double)(typename Acc<Ti>::type)in[(int64_t)f * N + e] * mul[f];
    out[(int64_t)f * N + e] = (To)(typename Acc<To>::type)v;
}

__global__ void k_f16_mul_t(const double* __restrict__ sumsq, int nf, int64_t n, double sig_u, double sig_p,
                            double target, double* __restrict__ mul) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t = 0;
    for (int f = 0; f < nf; ++f) {
        const double sg = f + 1 < nf ? sig_u : sig_p;
        t += sg * sg * sumsq[f];
    }
    const double rms = sqrt(t / (double)n);
    const double g = (rms > 0 && isfinite(rms)) ? target / rms : 1.0;
    for (int f = 0; f < nf; ++f) {
        const double sg = f + 1 < nf ? sig_u : sig_p;
        mul[f] = g * sg;
        mul[nf + f] = sg / g;
    }
}

// y = A x, A dense m x m row major; one wavefront per row.
__global__ __launch_bounds__(256) void k_dense_matvec_t(const double* __restrict__ A, int64_t m,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const double* a = A + row * m;
    double acc = 0;
    for (int64_t c = lane; c < m; c += 64) acc += a[c] * x[c];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) y[row] = acc;
}

// buoyancy load: b_{d-1}(v) = -rho sum_{T ni v, buoyant} |T| / (d+1)
template <int D>
__global__ __launch_bounds__(256) void k_buoyancy_bulk(LevelView L, const uint8_t* __restrict__ flag,
                                                       double rho, double vol, double* __restrict__ b) {
    constexpr int NS = KuhnTables<D>::NS;
    int i, j, k;
    if (!interior_vertex<D>(L, blockIdx.x, i, j, k)) return;
    const int64_t v = i + j * L.sy + k * L.sz;
    const int ph = L.vphase[v];
    if (ph == SPECIAL) return;
    b[(int64_t)(D - 1) * L.N + v] = flag[ph] ? -rho * NS * vol / (D + 1) : 0.0;
}

template <int D>
__global__ __launch_bounds__(256) void k_buoyancy_special(LevelView L, const uint8_t* __restrict__ flag,
                                                          double rho, double vol, double* __restrict__ b) {
    constexpr int NS = KuhnTables<D>::NS;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= L.spec_off[D + 1]) return;
    const int64_t v = L.spec[s];
    int ijk[3];
    vertex_ijk<D>(L, v, ijk);
    double acc = 0;
    for (int sl = 0; sl < NS; ++sl) {
        const int ph = L.spec_eph[s * NS + sl];
        if (ph != OUTSIDE && flag[ph]) acc += vol;
    }
    b[(int64_t)(D - 1) * L.N + v] = vel_fixed<D>(L, ijk, D - 1) ? 0.0 : -rho * acc / (D + 1);
}

// Load of a nodal body force: b_k = M f_k, M the P1 mass matrix (entries
// |T| (1 + delta_ab) / ((d+1)(d+2)) on each simplex T), one vertex per
// thread summing over the incident elements that lie in the domain.
template <int D>
__global__ __launch_bounds__(256) void k_nodal_force(LevelView L, const double* __restrict__ f,
                                                     double vol, double* __restrict__ b) {
    constexpr int NS = KuhnTables<D>::NS;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= L.N) return;
    int ijk[3];
    vertex_ijk<D>(L, v, ijk);
    double acc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] = 0;
    static_for<0, NS>([&](auto slc) {
        constexpr int sl = decltype(slc)::value;
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int c = ijk[a] + Kuhn<D>::T.slot_cell[sl][a];
            in = in && c >= 0 && c < L.n;
        }
        if (!in) return;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double sum = f[(int64_t)k * L.N + v];          // the diagonal's second half
            static_for<0, D + 1>([&](auto bc) {
                constexpr int o = Kuhn<D>::T.slot_nb[sl][decltype(bc)::value];
                sum += f[(int64_t)k * L.N + v + nb_lin<D>(L, o)];
            });
            acc[k] += sum;
        }
    });
    const double w = vol / ((D + 1) * (D + 2));
#pragma unroll
    for (int k = 0; k < D; ++k) b[(int64_t)k * L.N + v] = vel_fixed<D>(L, ijk, k) ? 0.0 : w * acc[k];
    b[(int64_t)D * L.N + v] = 0.0;
}

// ----------------------------------------------------------------------------
// launchers

static inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

// storage type T of a precision code, then the statements
#define ISS_BY_PREC(prec, ...)                                \
    switch (prec) {                                           \
        case PREC_F64: { using T = double; __VA_ARGS__; }     \
        break;                                                \
        case PREC_F32: { using T = float; __VA_ARGS__; }      \
        break;                                                \
        case PREC_BF16: { using T = __bf16; __VA_ARGS__; }    \
        break;                                                \
        case PREC_F16: { using T = _Float16; __VA_ARGS__; }   \
        break;                                                \
        default: return hipErrorInvalidValue;                 \
    }

hipError_t upload_tables(int dim, const void* t64, size_t bytes64, const void* t32, size_t bytes32) {
    hipError_t e;
    if (dim == 3) {
        if (bytes64 != sizeof(ElemTables<3, double>) || bytes32 != sizeof(ElemTables<3, float>))
            return hipErrorInvalidValue;
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_e3d), t64, bytes64);
        if (e != hipSuccess) return e;
        return hipMemcpyToSymbol(HIP_SYMBOL(g_e3f), t32, bytes32);
    }
    if (bytes64 != sizeof(ElemTables<2, double>) || bytes32 != sizeof(ElemTables<2, float>))
        return hipErrorInvalidValue;
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_e2d), t64, bytes64);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(g_e2f), t32, bytes32);
}

static inline int64_t special_blocks(int64_t ns, int wg = 256) { return (ns + wg - 1) / wg; }

// host-side launch counter of the stencil kernels (iss_launch_counts)
static inline void counted(const LevelView& L, int kind) {
    if (L.launch_count) ++L.launch_count[kind];
}

template <int D, int F, int BLK, int MODE, typename T>
static hipError_t apply_t(const LevelView& L, const T* x, const T* b, T* y, hipStream_t s) {
    const int64_t nb = interior_blocks<D>(L.n);
    if constexpr (D == 3) {
        if (L.n > L.merge_max_n && L.n >= 2) {      // large levels: LDS z march
            const ZTileGrid zg = ztile_grid(L.n);
            hipLaunchKernelGGL((k_apply_z<F, BLK, MODE, T>), dim3((unsigned)(NXCD * zg.gx * zg.gys * zg.gz)), dim3(256),
                               0, s, L, zg, x, b, y);
            counted(L, ISS_L_APPLY_TILED);
        } else if (nb > 0) {
            hipLaunchKernelGGL((k_apply_bulk<D, F, BLK, MODE, T>), dim3((unsigned)nb), dim3(BX, BY), 0, s,
                               L, x, b, y);
            counted(L, ISS_L_APPLY_BULK);
        }
    } else if (nb > 0) {
        hipLaunchKernelGGL((k_apply_bulk<D, F, BLK, MODE, T>), dim3((unsigned)nb), dim3(BX, BY), 0, s,
                           L, x, b, y);
        counted(L, ISS_L_APPLY_BULK);
    }
    const int64_t ns = special_blocks(L.spec_off[D + 1]);
    if (ns > 0)
        hipLaunchKernelGGL((k_apply_special<D, F, BLK, MODE, T>), dim3((unsigned)ns), dim3(256), 0, s,
                           L, x, b, y);
    return hipGetLastError();
}

template <int D, typename T>
static hipError_t apply_d(const LevelView& L, int form, int block, int mode, const T* x, const T* b,
                          T* y, hipStream_t s) {
#define ISS_AP(F, BL, MO) \
    if (form == F && block == BL && mode == MO) return apply_t<D, F, BL, MO, T>(L, x, b, y, s);
    ISS_AP(0, 0, 0) ISS_AP(0, 0, 1) ISS_AP(0, 1, 0) ISS_AP(0, 1, 1)
    ISS_AP(1, 0, 0) ISS_AP(1, 0, 1) ISS_AP(1, 1, 0) ISS_AP(1, 1, 1)
    ISS_AP(2, 0, 0) ISS_AP(2, 0, 1) ISS_AP(2, 1, 0) ISS_AP(2, 1, 1)
#undef ISS_AP
    return hipErrorInvalidValue;
}

hipError_t k_apply(const LevelView& L, int form, int block, int mode, int prec, const void* x,
                   const void* b, void* y, hipStream_t s) {
    ISS_BY_PREC(prec,
        if (L.dim == 3) return apply_d<3, T>(L, form, block, mode, (const T*)x, (const T*)b, (T*)y, s);
        return apply_d<2, T>(L, form, block, mode, (const T*)x, (const T*)b, (T*)y, s))
    return hipErrorInvalidValue;
}

static inline unsigned blocks256(int64_t threads) { return (unsigned)((threads + 255) / 256); }


// One Uzawa step (eq. Uzawa_smooth) on split-layout vectors: symmetric
// velocity sweep (forward colours 0..d, backward d..0, the repeated colour d
// skipped where it is a no-op; bulk then special launch per colour), then the pressure forward sweep on C from delta = 0
// (colour 0 inside the s pass), p += omega delta.  ws holds d + 1 split
// fields: g = f - B^T p in fields 0..d-1 during the velocity sweep,
// s = B u - C p - g in field 0 and delta in field d during the pressure
// sweep.  Each step leaves delta cleared; the first step of a sequence
// (first_step) clears it itself, so a sequence never depends on what an
// earlier call left in ws.
template <int D, int F, typename T>
static hipError_t smooth_t(const LevelView& L, double omega, T* xs, const T* bs, T* ws, bool first_step,
                           hipStream_t s, PhaseTimer* tm) {
    const int64_t ba = split_slab_blocks<D>(L.n, (L.n - 1) / (D + 1) + 1);   // grouped (velocity rhs)
    const int64_t bp = split_slab_blocks<D>(L.n, L.Rp);                      // one vertex per thread
    const int64_t bc = split_slab_blocks<D>(L.n, (L.n - 1) / (D + 1) + 1);
    T* g = ws;
    T* sres = ws;
    T* delta = ws + (int64_t)D * L.Ns;
    const bool merge = L.n <= L.merge_max_n;     // one launch per colour phase
    // LDS-tiled right-hand-side passes on the large 3D levels
    const bool ztiled = D == 3 && !merge && L.n >= 2;
    const ZTileGrid zg = ztile_grid(L.n);
    const unsigned bz = (unsigned)(NXCD * zg.gx * zg.gys * zg.gz);
    if (ztiled) {
        hipLaunchKernelGGL((k_vel_rhs_z<T>), dim3(bz), dim3(256), 0, s, L, zg, xs, bs, g);
        counted(L, ISS_L_VEL_RHS);
    } else if (ba > 0) {
        hipLaunchKernelGGL((k_vel_rhs_s<D, T>), dim3((unsigned)ba), dim3(256), 0, s, L, xs, bs, g);
        counted(L, ISS_L_VEL_RHS);
    }
    // The backward sweep starts with the colour the forward sweep ended
    // with.  Where every point-diagonal block is diagonal (gradient and
    // interface forms: the a_tr block of a vertex with itself is
    // mu |grad phi|^2 I), that phase repeats an exact solve of rows whose
    // neighbours have not changed, so it is a no-op in exact arithmetic and
    // is skipped (bulk rows would reproduce the same bits; special rows
    // would add a rounding-level correction).  The strain form's coupled
    // block with the reversed component order is not idempotent: it runs.
    constexpr int first_bwd = (F == FORM_STRAIN) ? 0 : 1;
    if (tm) tm->used = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int cc = (pass == 0 ? 0 : first_bwd); cc <= D; ++cc) {
            const int c = pass == 0 ? cc : D - cc;
            const int64_t ns = special_blocks(L.spec_off[c + 1] - L.spec_off[c]);
            const int64_t nsw = special_blocks(L.spec_off[c + 1] - L.spec_off[c], SPEC_WG);
            // the special-only launch covers the interior rows alone under no-slip
            const int64_t nsv = special_blocks(L.spec_off[c + 1] - (L.freeslip ? L.spec_off[c] : L.spec_mid[c]),
                                               SPEC_WG);
            const int tq = tm ? tm->used++ : 0;
            if (tm) (void)hipEventRecord(tm->begin[tq], s);
            if (merge && bc > 0 && ns > 0) {
                if (pass == 0)
                    hipLaunchKernelGGL((k_gs_vel_m<D, F, false, T>), dim3((unsigned)(4 * bc + nsw)), dim3(64), 0, s, L, c,
                                       xs, g, bs, bc);
                else
                    hipLaunchKernelGGL((k_gs_vel_m<D, F, true, T>), dim3((unsigned)(4 * bc + nsw)), dim3(64), 0, s, L, c,
                                       xs, g, bs, bc);
                counted(L, ISS_L_GS_VEL_MERGED);
                if (tm) (void)hipEventRecord(tm->end[tq], s);
            } else {
                if (bc > 0) {
                    if (pass == 0)
                        hipLaunchKernelGGL((k_gs_vel_s<D, F, false, T>), dim3((unsigned)bc), dim3(256), 0, s, L, c, xs, g);
                    else
                        hipLaunchKernelGGL((k_gs_vel_s<D, F, true, T>), dim3((unsigned)bc), dim3(256), 0, s, L, c, xs, g);
                    counted(L, ISS_L_GS_VEL_BULK);
                }
                if (tm) (void)hipEventRecord(tm->end[tq], s);
                if (nsv > 0) {
                    if (pass == 0)
                        hipLaunchKernelGGL((k_gs_vel_special_s<D, F, false, T>), dim3((unsigned)nsv), dim3(SPEC_WG), 0, s, L,
                                           c, xs, bs);
                    else
                        hipLaunchKernelGGL((k_gs_vel_special_s<D, F, true, T>), dim3((unsigned)nsv), dim3(SPEC_WG), 0, s, L,
                                           c, xs, bs);
                    counted(L, ISS_L_GS_VEL_SPECIAL);
                }
            }
        }
    }
    if (first_step)
        hipLaunchKernelGGL((k_fill_t<T>), grid1(L.Ns), dim3(256), 0, s, delta, L.Ns, (typename Acc<T>::type)0);
    for (int c = 0; c <= D; ++c) {
        const int64_t ns = special_blocks(L.spec_off[c + 1] - L.spec_off[c]);
        const int64_t nsw = special_blocks(L.spec_off[c + 1] - L.spec_off[c], SPEC_WG);
        if (c == 0) {
            // s pass with colour 0 folded in
            const int64_t nb = ba > 0 ? bp : 0;
            if (merge && nb + ns > 0) {
                hipLaunchKernelGGL((k_p_rhs_s<D, T>), dim3((unsigned)(4 * nb + nsw)), dim3(64), 0, s, L, xs, bs,
                                   sres, delta, nb);
                counted(L, ISS_L_P_RHS_MERGED);
                continue;
            }
            if (ztiled) {
                hipLaunchKernelGGL((k_p_rhs_z<T>), dim3(bz), dim3(256), 0, s, L, zg, xs, bs, sres, delta);
                counted(L, ISS_L_P_RHS_GROUPED);
            } else if (ba > 0) {
                hipLaunchKernelGGL((k_p_rhs_g<D, T>), dim3((unsigned)ba), dim3(256), 0, s, L, xs, bs, sres, delta);
                counted(L, ISS_L_P_RHS_GROUPED);
            }
        } else if (merge && bc > 0 && ns > 0) {
            hipLaunchKernelGGL((k_gs_p_m<D, T>), dim3((unsigned)(4 * bc + nsw)), dim3(64), 0, s, L, c, sres, xs, bs,
                               delta, bc);
            counted(L, ISS_L_GS_P_MERGED);
            continue;
        } else if (bc > 0) {
            hipLaunchKernelGGL((k_gs_p_s<D, T>), dim3((unsigned)bc), dim3(256), 0, s, L, c, sres, delta);
            counted(L, ISS_L_GS_P_BULK);
        }
        if (ns > 0 && L.spec_off[c + 1] - L.spec_off[c] > L.spec_wide_min) {
            hipLaunchKernelGGL((k_gs_p_special_s<D, T, 256>), dim3((unsigned)ns), dim3(256), 0, s, L, c, xs, bs, delta);
            counted(L, ISS_L_GS_P_SPECIAL_WIDE);
        } else if (ns > 0) {
            hipLaunchKernelGGL((k_gs_p_special_s<D, T, SPEC_WG>), dim3((unsigned)nsw), dim3(SPEC_WG), 0, s, L, c, xs,
                               bs, delta);
            counted(L, ISS_L_GS_P_SPECIAL);
        }
    }
    hipLaunchKernelGGL((k_axpy_clear<T>), grid1(L.Ns), dim3(256), 0, s, xs + (int64_t)D * L.Ns, delta,
                       (typename Acc<T>::type)omega, L.Ns);
    return hipGetLastError();
}

template <int D, typename T>
static hipError_t smooth_d(const LevelView& L, int form, double omega, T* xs, const T* bs, T* ws,
                           bool first_step, hipStream_t s, PhaseTimer* tm) {
    if (form == FORM_GRADIENT) return smooth_t<D, 0, T>(L, omega, xs, bs, ws, first_step, s, tm);
    if (form == FORM_STRAIN) return smooth_t<D, 1, T>(L, omega, xs, bs, ws, first_step, s, tm);
    if (form == FORM_INTERFACE) return smooth_t<D, 2, T>(L, omega, xs, bs, ws, first_step, s, tm);
    return hipErrorInvalidValue;
}

hipError_t k_smooth_step(const LevelView& L, int form, int prec, double omega, void* xs, const void* bs,
                         void* ws, bool first_step, hipStream_t s, PhaseTimer* tm) {
    ISS_BY_PREC(prec,
        if (L.dim == 3) return smooth_d<3, T>(L, form, omega, (T*)xs, (const T*)bs, (T*)ws, first_step, s, tm);
        return smooth_d<2, T>(L, form, omega, (T*)xs, (const T*)bs, (T*)ws, first_step, s, tm))
    return hipErrorInvalidValue;
}

template <int D, typename T>
static void split_t(const LevelView& L, int nf, const T* in, T* out, int dir, hipStream_t s) {
    if (dir == SPLIT_PACK)
        hipLaunchKernelGGL((k_pack_t<D, T>), dim3(blocks256(L.Ns), nf), dim3(256), 0, s, L, in, out);
    else
        hipLaunchKernelGGL((k_unpack_t<D, T>), dim3(blocks256(L.N), nf), dim3(256), 0, s, L, in, out);
}

hipError_t k_split(const LevelView& L, int prec, int nf, const void* in, void* out, int dir, hipStream_t s) {
    if (nf <= 0) return hipSuccess;
    ISS_BY_PREC(prec,
        if (L.dim == 3) split_t<3, T>(L, nf, (const T*)in, (T*)out, dir, s);
        else split_t<2, T>(L, nf, (const T*)in, (T*)out, dir, s))
    return hipGetLastError();
}

hipError_t k_restrict(const LevelView& Lf, const LevelView& Lc, int prec, const void* rf, void* rc,
                      hipStream_t s) {
    ISS_BY_PREC(prec,
        if (Lf.dim == 3) hipLaunchKernelGGL((k_restrict_t<3, T>), grid1(Lc.N), dim3(256), 0, s, Lf, Lc, (const T*)rf, (T*)rc);
        else hipLaunchKernelGGL((k_restrict_t<2, T>), grid1(Lc.N), dim3(256), 0, s, Lf, Lc, (const T*)rf, (T*)rc))
    return hipGetLastError();
}

hipError_t k_prolong_add(const LevelView& Lf, const LevelView& Lc, int prec, const void* ec, void* xf,
                         hipStream_t s) {
    ISS_BY_PREC(prec,
        if (Lf.dim == 3) hipLaunchKernelGGL((k_prolong_t<3, T>), grid1(Lf.N), dim3(256), 0, s, Lf, Lc, (const T*)ec, (T*)xf);
        else hipLaunchKernelGGL((k_prolong_t<2, T>), grid1(Lf.N), dim3(256), 0, s, Lf, Lc, (const T*)ec, (T*)xf))
    return hipGetLastError();
}

hipError_t k_fill(int prec, void* x, int64_t n, double value, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    ISS_BY_PREC(prec,
        hipLaunchKernelGGL((k_fill_t<T>), grid1(n), dim3(256), 0, s, (T*)x, n, (typename Acc<T>::type)value))
    return hipGetLastError();
}

hipError_t k_convert(int prec_in, const void* in, int prec_out, void* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // one side is FP64 (the Krylov vectors), the other any storage type
    if (prec_in == PREC_F64) {
        ISS_BY_PREC(prec_out,
            hipLaunchKernelGGL((k_convert_t<double, T>), grid1(n), dim3(256), 0, s, (const double*)in, (T*)out, n))
    } else if (prec_out == PREC_F64) {
        ISS_BY_PREC(prec_in,
            hipLaunchKernelGGL((k_convert_t<T, double>), grid1(n), dim3(256), 0, s, (const T*)in, (double*)out, n))
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t k_field_sumsq(int prec, const void* x, int64_t N, int nf, double* partial, double* out,
                         hipStream_t s) {
    const int nblk = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (N + 255) / 256));
    ISS_BY_PREC(prec,
        hipLaunchKernelGGL((k_sumsq_partial<T>), dim3(nblk), dim3(256), 0, s, (const T*)x, N, nf, partial))
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nblk, nf, out);
    return hipGetLastError();
}

hipError_t k_field_sum(const double* x, int64_t N, double* partial, double* out, hipStream_t s) {
    const int nblk = (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (N + 255) / 256));
    hipLaunchKernelGGL((k_sumsq_partial<double, false>), dim3(nblk), dim3(256), 0, s, x, N, 1, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nblk, 1, out);
    return hipGetLastError();
}

// x -= sum[0] / n (sum on the device: no host round trip)
__global__ __launch_bounds__(256) void k_sub_mean_t(double* __restrict__ x, int64_t n,
                                                    const double* __restrict__ sum) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) x[e] -= sum[0] / (double)n;
}

hipError_t k_sub_mean(double* x, int64_t n, const double* sum, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_mean_t, grid1(n), dim3(256), 0, s, x, n, sum);
    return hipGetLastError();
}

hipError_t k_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n, double* partial,
                      double* out, hipStream_t s, int with_self) {
    // partial holds 1024 * 64 doubles: at most 65536 / (k + 1) blocks per vector
    const int kk = k + with_self;
    const int64_t cap = std::max<int64_t>(1, 65536 / std::max(1, kk));
    const int nblk = (int)std::min<int64_t>(std::min<int64_t>(1024, cap), std::max<int64_t>(1, (n + 255) / 256));
    const int tiles = (kk + MD_TILE - 1) / MD_TILE;
    hipLaunchKernelGGL(k_multidot_partial, dim3(tiles, nblk), dim3(256), 0, s, V, ldv, k, w, n, partial, with_self);
    hipLaunchKernelGGL(k_sum_slots, dim3(kk), dim3(256), 0, s, partial, nblk, out);
    return hipGetLastError();
}

// even length and leading dimension, 16-byte aligned vectors: the Krylov
// kernels may read two doubles per lane
static inline bool pair_aligned(int64_t n, int64_t ldv, const void* p, const void* q, const void* r) {
    auto al = [](const void* x) { return ((uintptr_t)x & 15) == 0; };
    return n % 2 == 0 && ldv % 2 == 0 && al(p) && al(q) && al(r);
}

hipError_t k_dots2(const double* V, int64_t ldv, int k, const double* a, const double* b, int64_t n,
                   double* partial, double* out, hipStream_t s) {
    const int slots = 2 * k + 3;
    const int nblk = (int)std::min<int64_t>(std::min<int64_t>(1024, 65536 / slots),
                                            std::max<int64_t>(1, (n + 255) / 256));
    const int tiles = std::max(1, (k + MD_TILE - 1) / MD_TILE);
    if (pair_aligned(n, ldv, V, a, b))
        hipLaunchKernelGGL(k_dots2_partial<2>, dim3(tiles, nblk), dim3(256), 0, s, V, ldv, k, a, b, n, partial);
    else
        hipLaunchKernelGGL(k_dots2_partial<1>, dim3(tiles, nblk), dim3(256), 0, s, V, ldv, k, a, b, n, partial);
    hipLaunchKernelGGL(k_sum_slots, dim3(slots), dim3(256), 0, s, partial, nblk, out);
    return hipGetLastError();
}

hipError_t k_dcgs_update(double* V, int64_t ldv, int k, const double* c, const double* d, const double* w,
                         double inv_alpha, double ecoef, double inv_s, int64_t n, hipStream_t s) {
    if (pair_aligned(n, ldv, V, w, w))
        hipLaunchKernelGGL(k_dcgs_update_t<2>, grid1((n + 1) / 2), dim3(256), 0, s, V, ldv, k, c, d, w,
                           inv_alpha, ecoef, inv_s, n);
    else
        hipLaunchKernelGGL(k_dcgs_update_t<1>, grid1(n), dim3(256), 0, s, V, ldv, k, c, d, w, inv_alpha,
                           ecoef, inv_s, n);
    return hipGetLastError();
}

hipError_t k_multiaxpy(double* y, const double* X, int64_t ldx, int k, const double* c, double alpha,
                       int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_multiaxpy_t, grid1(n), dim3(256), 0, s, y, X, ldx, k, c, alpha, n);
    return hipGetLastError();
}

hipError_t k_scale(double* y, double a, const double* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_t, grid1(n), dim3(256), 0, s, y, a, x, n);
    return hipGetLastError();
}

hipError_t k_axpby(double* y, double a, const double* x, double b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby_t, grid1(n), dim3(256), 0, s, y, a, x, b, n);
    return hipGetLastError();
}

hipError_t k_gather(int prec, const void* x, const int32_t* idx, int64_t m, double* out, hipStream_t s,
                    FieldMul fm) {
    ISS_BY_PREC(prec,
        hipLaunchKernelGGL((k_gather_t<T>), grid1(m), dim3(256), 0, s, (const T*)x, idx, m, out, fm))
    return hipGetLastError();
}

hipError_t k_scatter(int prec, const double* in, const int32_t* idx, int64_t m, void* x, hipStream_t s,
                     FieldMul fm) {
    ISS_BY_PREC(prec,
        hipLaunchKernelGGL((k_scatter_t<T>), grid1(m), dim3(256), 0, s, in, idx, m, (T*)x, fm))
    return hipGetLastError();
}

hipError_t k_scale_convert(int prec, int dir, const void* in, void* out, int64_t N, int nf, const double* mul,
                           hipStream_t s) {
    if (N <= 0 || nf <= 0) return hipSuccess;
    const dim3 g((unsigned)((N + 255) / 256), (unsigned)nf);
    if (dir == 0) {
        ISS_BY_PREC(prec,
            hipLaunchKernelGGL((k_scale_convert_t<double, T>), g, dim3(256), 0, s, (const double*)in, (T*)out, N, mul))
    } else {
        ISS_BY_PREC(prec,
            hipLaunchKernelGGL((k_scale_convert_t<T, double>), g, dim3(256), 0, s, (const T*)in, (double*)out, N, mul))
    }
    return hipGetLastError();
}

hipError_t k_f16_multipliers(const double* sumsq, int nf, int64_t n, double sig_u, double sig_p, double target,
                             double* mul, hipStream_t s) {
    hipLaunchKernelGGL(k_f16_mul_t, dim3(1), dim3(64), 0, s, sumsq, nf, n, sig_u, sig_p, target, mul);
    return hipGetLastError();
}

hipError_t k_dense_matvec(const double* A, int64_t m, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_matvec_t, grid1(m, 4), dim3(256), 0, s, A, m, x, y);
    return hipGetLastError();
}

hipError_t k_rhs_buoyancy(const LevelView& L, const uint8_t* flag, double rho, double vol, double* b,
                          hipStream_t s) {
    const int D = L.dim;
    const int64_t nb = D == 3 ? interior_blocks<3>(L.n) : interior_blocks<2>(L.n);
    const int64_t ns = L.spec_off[D + 1];
    if (D == 3) {
        if (nb > 0) hipLaunchKernelGGL(k_buoyancy_bulk<3>, dim3((unsigned)nb), dim3(BX, BY), 0, s, L, flag, rho, vol, b);
        if (ns > 0) hipLaunchKernelGGL(k_buoyancy_special<3>, grid1(ns), dim3(256), 0, s, L, flag, rho, vol, b);
    } else {
        if (nb > 0) hipLaunchKernelGGL(k_buoyancy_bulk<2>, dim3((unsigned)nb), dim3(BX, BY), 0, s, L, flag, rho, vol, b);
        if (ns > 0) hipLaunchKernelGGL(k_buoyancy_special<2>, grid1(ns), dim3(256), 0, s, L, flag, rho, vol, b);
    }
    return hipGetLastError();
}

hipError_t k_rhs_nodal_force(const LevelView& L, const double* f, double vol, double* b, hipStream_t s) {
    if (L.dim == 3) hipLaunchKernelGGL(k_nodal_force<3>, grid1(L.N), dim3(256), 0, s, L, f, vol, b);
    else hipLaunchKernelGGL(k_nodal_force<2>, grid1(L.N), dim3(256), 0, s, L, f, vol, b);
    return hipGetLastError();
}

}  // namespace iss
