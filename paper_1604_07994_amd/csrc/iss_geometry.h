// Compile-time geometry of the Kuhn (Freudenthal) lattice.
//
// The uniformly refined cube macro meshes of the paper (six tetrahedra per
// cube, Sec. 4; Bey refinement, Sec. 3 remark) are Kuhn lattices: every
// lattice cell holds the d! simplices x0, x0+e_pi(0), x0+e_pi(0)+e_pi(1),
// ..., x0+(1..1), one per permutation pi.  Around a vertex these tables
// give
//   * the stencil footprint: the centre and +-w for the 2^d - 1 nonzero
//     0/1 vectors w (15 points in 3D, 7 in 2D),
//   * the incident elements ("slots"): element type pi and local index a of
//     the vertex in it (d! (d+1) slots: 24 in 3D, 6 in 2D), and for each
//     slot the footprint index of each element vertex.
// Everything is constexpr so that fully unrolled kernel loops index
// register arrays with constants.
#pragma once

namespace iss {

template <int D> struct Kuhn;

template <int D>
struct KuhnTables {
    static constexpr int NB = (D == 3) ? 15 : 7;              // footprint
    static constexpr int NT = (D == 3) ? 6 : 2;               // element types
    static constexpr int NS = NT * (D + 1);                   // slots
    int off[NB][3];          // footprint offsets (z = 0 in 2D)
    int type_vert[NT][D + 1][3];   // Kuhn simplex vertices of each type
    int slot_type[NS];
    int slot_loc[NS];
    int slot_nb[NS][D + 1];  // footprint index of each element vertex
    int slot_cell[NS][3];    // cell origin relative to the vertex
};

namespace detail {

template <int D>
constexpr int find_off(const KuhnTables<D>& t, int x, int y, int z) {
    for (int o = 0; o < KuhnTables<D>::NB; ++o)
        if (t.off[o][0] == x && t.off[o][1] == y && t.off[o][2] == z) return o;
    return -1;
}

template <int D>
constexpr KuhnTables<D> make_tables() {
    KuhnTables<D> t{};
    // footprint: centre, then +w, -w for w = e1, e2, (e3), e1+e2, (e1+e3,
    // e2+e3, e1+e2+e3)
    int ws[7][3] = {};
    int nw = 0;
    if (D == 3) {
        int w3[7][3] = {{1,0,0},{0,1,0},{0,0,1},{1,1,0},{1,0,1},{0,1,1},{1,1,1}};
        for (int i = 0; i < 7; ++i) for (int a = 0; a < 3; ++a) ws[i][a] = w3[i][a];
        nw = 7;
    } else {
        int w2[3][3] = {{1,0,0},{0,1,0},{1,1,0}};
        for (int i = 0; i < 3; ++i) for (int a = 0; a < 3; ++a) ws[i][a] = w2[i][a];
        nw = 3;
    }
    for (int a = 0; a < 3; ++a) t.off[0][a] = 0;
    for (int i = 0; i < nw; ++i)
        for (int a = 0; a < 3; ++a) {
            t.off[1 + 2 * i][a] = ws[i][a];
            t.off[2 + 2 * i][a] = -ws[i][a];
        }
    // element types: permutations in lexicographic order
    int perms3[6][3] = {{0,1,2},{0,2,1},{1,0,2},{1,2,0},{2,0,1},{2,1,0}};
    int perms2[2][3] = {{0,1,0},{1,0,0}};
    for (int ty = 0; ty < KuhnTables<D>::NT; ++ty) {
        int cur[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) t.type_vert[ty][0][a] = 0;
        for (int s = 0; s < D; ++s) {
            int ax = (D == 3) ? perms3[ty][s] : perms2[ty][s];
            cur[ax] += 1;
            for (int a = 0; a < 3; ++a) t.type_vert[ty][s + 1][a] = cur[a];
        }
    }
    // slots: (type, local index)
    int s = 0;
    for (int ty = 0; ty < KuhnTables<D>::NT; ++ty)
        for (int loc = 0; loc <= D; ++loc) {
            t.slot_type[s] = ty;
            t.slot_loc[s] = loc;
            for (int a = 0; a < 3; ++a) t.slot_cell[s][a] = -t.type_vert[ty][loc][a];
            for (int b = 0; b <= D; ++b)
                t.slot_nb[s][b] = find_off<D>(t,
                    t.type_vert[ty][b][0] - t.type_vert[ty][loc][0],
                    t.type_vert[ty][b][1] - t.type_vert[ty][loc][1],
                    t.type_vert[ty][b][2] - t.type_vert[ty][loc][2]);
            ++s;
        }
    return t;
}

}  // namespace detail

template <> struct Kuhn<3> {
    static constexpr KuhnTables<3> T = detail::make_tables<3>();
};
template <> struct Kuhn<2> {
    static constexpr KuhnTables<2> T = detail::make_tables<2>();
};

// Barycentric gradients of the unit Kuhn simplices.  For the simplex
// 0, e_p0, e_p0 + e_p1, ... the coordinates are lambda_0 = 1 - x_p0,
// lambda_s = x_p(s-1) - x_ps, lambda_d = x_p(d-1), so every gradient is an
// integer vector with entries in {-1, 0, 1} and the element volume is 1/d!.
// The element matrices below are therefore exact rationals known at compile
// time; the special-vertex kernels fold them into immediates instead of
// reading tables.
template <int D>
struct KuhnGrads {
    int g[KuhnTables<D>::NT][D + 1][3];
};

namespace detail {
template <int D>
constexpr KuhnGrads<D> make_grads() {
    KuhnGrads<D> r{};
    constexpr auto& K = Kuhn<D>::T;
    for (int ty = 0; ty < KuhnTables<D>::NT; ++ty) {
        int ax[3] = {0, 0, 0};
        for (int s = 0; s < D; ++s)
            for (int a = 0; a < 3; ++a)
                if (K.type_vert[ty][s + 1][a] - K.type_vert[ty][s][a] == 1) ax[s] = a;
        for (int v = 0; v <= D; ++v)
            for (int a = 0; a < 3; ++a) r.g[ty][v][a] = 0;
        r.g[ty][0][ax[0]] = -1;
        for (int s = 1; s < D; ++s) {
            r.g[ty][s][ax[s - 1]] += 1;
            r.g[ty][s][ax[s]] -= 1;
        }
        r.g[ty][D][ax[D - 1]] = 1;
    }
    return r;
}
}  // namespace detail

template <int D> struct KGrad { static constexpr KuhnGrads<D> G = detail::make_grads<D>(); };

// unit-lattice element volume 1/d!
template <int D> constexpr double kuhn_volume() { return D == 3 ? 1.0 / 6.0 : 0.5; }

// integer part of the element matrices (times the volume): test phi_a e_l,
// trial phi_b e_k of element type ty
template <int D>
constexpr int kg_dot(int ty, int a, int b) {
    int s = 0;
    for (int q = 0; q < D; ++q) s += KGrad<D>::G.g[ty][a][q] * KGrad<D>::G.g[ty][b][q];
    return s;
}
// form 0: (grad, grad); 1: 2 (sym grad, sym grad); 2: 1 minus (div, div)
template <int D>
constexpr int kg_visc(int form, int ty, int a, int l, int b, int k) {
    const auto& g = KGrad<D>::G.g[ty];
    const int lap = (k == l) ? kg_dot<D>(ty, a, b) : 0;
    if (form == 0) return lap;
    const int sym = lap + g[b][l] * g[a][k];
    if (form == 1) return sym;
    return sym - g[b][k] * g[a][l];
}

// Integer parts of the stencils of an isoviscous interior vertex (sums of
// the element entries over the incident elements): the divergence row B
// (times -|T|/(d+1)), its transpose B^T (same factor) and C (times |T|).
template <int D>
constexpr int sdiv_int(int k, int o) {
    constexpr auto& K = Kuhn<D>::T;
    int s = 0;
    for (int sl = 0; sl < KuhnTables<D>::NS; ++sl)
        for (int b = 0; b <= D; ++b)
            if (K.slot_nb[sl][b] == o) s += KGrad<D>::G.g[K.slot_type[sl]][b][k];
    return s;
}
template <int D>
constexpr int sbt_int(int l, int o) {
    constexpr auto& K = Kuhn<D>::T;
    int s = 0;
    for (int sl = 0; sl < KuhnTables<D>::NS; ++sl)
        for (int b = 0; b <= D; ++b)
            if (K.slot_nb[sl][b] == o) s += KGrad<D>::G.g[K.slot_type[sl]][K.slot_loc[sl]][l];
    return s;
}
template <int D>
constexpr int sc_int(int o) {
    constexpr auto& K = Kuhn<D>::T;
    int s = 0;
    for (int sl = 0; sl < KuhnTables<D>::NS; ++sl)
        for (int b = 0; b <= D; ++b)
            if (K.slot_nb[sl][b] == o) s += kg_dot<D>(K.slot_type[sl], K.slot_loc[sl], b);
    return s;
}
// integer part (times |T|) of the viscous stencil of an isoviscous interior
// vertex, viscosity 1: block (l, k) at footprint offset o, form as kg_visc
template <int D>
constexpr int svis_int(int form, int l, int k, int o) {
    constexpr auto& K = Kuhn<D>::T;
    int s = 0;
    for (int sl = 0; sl < KuhnTables<D>::NS; ++sl)
        for (int b = 0; b <= D; ++b)
            if (K.slot_nb[sl][b] == o) s += kg_visc<D>(form, K.slot_type[sl], K.slot_loc[sl], l, b, k);
    return s;
}
// footprint index of the offset (dx, dy, dz), or -1
template <int D>
constexpr int off_index(int dx, int dy, int dz) {
    return detail::find_off<D>(Kuhn<D>::T, dx, dy, dz);
}

// Floating-point element tables for the unit lattice (h = 1); per level the
// viscous block scales with h^(d-2), B with h^(d-1) and C with beta h^d.
//   Avis[f][type][a*D+l][b*D+k]: viscous form f (0 gradient, 1 strain,
//       2 a_tr) between test phi_a e_l and trial phi_b e_k, viscosity 1;
//   Bel[type][a][b*D+k]: -(div(phi_b e_k), lambda_a)_T;
//   Cel[type][a][b]: (grad lambda_b, grad lambda_a)_T;
// and the stencils of an isoviscous interior vertex (viscosity 1):
//   Svis[f][l][k][o], Sbt[l][o] (B^T), Sdiv[k][o] (B), Sc[o] (C / beta).
template <int D, typename C>
struct ElemTables {
    static constexpr int NB = KuhnTables<D>::NB;
    static constexpr int NT = KuhnTables<D>::NT;
    C Avis[3][NT][(D + 1) * D][(D + 1) * D];
    C Bel[NT][D + 1][(D + 1) * D];
    C Cel[NT][D + 1][D + 1];
    C Svis[3][D][D][NB];
    C Sbt[D][NB];
    C Sdiv[D][NB];
    C Sc[NB];
};

}  // namespace iss
