// Host side of the Stokes hot path: problem setup (element classification,
// interface lists, element tables, coarse factorisation), the multigrid and
// Krylov orchestration, and the C ABI declared in include/iss.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/iss.h"
#include "iss_internal.h"

using namespace iss;

// Scratch of iss_smooth_noalloc: the colour-split copies of x and b and the
// smoother's work fields.  One copy per GPU, held by the code object until
// the process ends.  In host code this name is a stand-in, not a device
// address: kernels get the address hipGetSymbolAddress returns for it.
static __device__ __align__(256) char scratch[ISS_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define ISS_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(ISS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// ----------------------------------------------------------------------------
// element tables of the unit lattice (h = 1)

// Barycentric gradients of a simplex: with M = [1 | X] (row i = [1, x_i]),
// lambda(x) = [1, x] M^{-1}; gradient of lambda_i = rows 1..d of column i.
template <int D>
void simplex_gradients(const int (&X)[D + 1][3], double (&g)[D + 1][D], double& vol) {
    double M[D + 1][D + 1], Inv[D + 1][D + 1];
    for (int i = 0; i <= D; ++i) {
        M[i][0] = 1.0;
        for (int a = 0; a < D; ++a) M[i][a + 1] = X[i][a];
        for (int j = 0; j <= D; ++j) Inv[i][j] = (i == j) ? 1.0 : 0.0;
    }
    double det = 1.0;
    for (int c = 0; c <= D; ++c) {          // Gauss-Jordan with partial pivoting
        int piv = c;
        for (int r = c + 1; r <= D; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (piv != c) {
            for (int j = 0; j <= D; ++j) { std::swap(M[c][j], M[piv][j]); std::swap(Inv[c][j], Inv[piv][j]); }
            det = -det;
        }
        const double d = M[c][c];
        det *= d;
        for (int j = 0; j <= D; ++j) { M[c][j] /= d; Inv[c][j] /= d; }
        for (int r = 0; r <= D; ++r) {
            if (r == c) continue;
            const double f = M[r][c];
            for (int j = 0; j <= D; ++j) { M[r][j] -= f * M[c][j]; Inv[r][j] -= f * Inv[c][j]; }
        }
    }
    for (int i = 0; i <= D; ++i)
        for (int a = 0; a < D; ++a) g[i][a] = Inv[a + 1][i];
    double fact = 1.0;
    for (int a = 2; a <= D; ++a) fact *= a;
    vol = std::fabs(det) / fact;
}

template <int D>
int build_tables(ElemTables<D, double>& t) {
    constexpr auto& K = Kuhn<D>::T;
    constexpr int NT = KuhnTables<D>::NT, NS = KuhnTables<D>::NS, NB = KuhnTables<D>::NB;
    std::memset(&t, 0, sizeof(t));
    for (int ty = 0; ty < NT; ++ty) {
        int X[D + 1][3];
        for (int b = 0; b <= D; ++b)
            for (int a = 0; a < 3; ++a) X[b][a] = K.type_vert[ty][b][a];
        double g[D + 1][D], vol;
        simplex_gradients<D>(X, g, vol);
        // the kernels use the exact integer gradients of iss_geometry.h
        if (std::fabs(vol - kuhn_volume<D>()) > 1e-15)
            return fail(ISS_E_INVAL, "geometry table: Kuhn simplex volume");
        for (int b = 0; b <= D; ++b)
            for (int q = 0; q < D; ++q)
                if (std::fabs(g[b][q] - KGrad<D>::G.g[ty][b][q]) > 1e-13)
                    return fail(ISS_E_INVAL, "geometry table: Kuhn gradients");
        for (int a = 0; a <= D; ++a)          // test vertex
            for (int b = 0; b <= D; ++b) {    // trial vertex
                double gg = 0;
                for (int q = 0; q < D; ++q) gg += g[a][q] * g[b][q];
                t.Cel[ty][a][b] = vol * gg;
                for (int l = 0; l < D; ++l)
                    for (int k = 0; k < D; ++k) {
                        // (mu grad(phi_b e_k), grad(phi_a e_l)) with mu = 1
                        const double lap = (k == l) ? vol * gg : 0.0;
                        // 2 sym(grad)(trial) : sym(grad)(test)
                        const double sym = lap + vol * g[b][l] * g[a][k];
                        // (div trial, div test)
                        const double dv = vol * g[b][k] * g[a][l];
                        t.Avis[FORM_GRADIENT][ty][a * D + l][b * D + k] = lap;
                        t.Avis[FORM_STRAIN][ty][a * D + l][b * D + k] = sym;
                        t.Avis[FORM_INTERFACE][ty][a * D + l][b * D + k] = sym - dv;
                    }
                // -(div(phi_b e_k), lambda_a) with int lambda_a = vol / (d+1)
                for (int k = 0; k < D; ++k) t.Bel[ty][a][b * D + k] = -vol / (D + 1) * g[b][k];
            }
    }
    // stencils of an interior vertex with all incident elements present
    for (int s = 0; s < NS; ++s) {
        const int ty = K.slot_type[s], a = K.slot_loc[s];
        for (int b = 0; b <= D; ++b) {
            const int o = K.slot_nb[s][b];
            if (o < 0) return fail(ISS_E_INVAL, "geometry table: element vertex outside footprint");
            for (int f = 0; f < 3; ++f)
                for (int l = 0; l < D; ++l)
                    for (int k = 0; k < D; ++k) t.Svis[f][l][k][o] += t.Avis[f][ty][a * D + l][b * D + k];
            for (int l = 0; l < D; ++l) t.Sbt[l][o] += t.Bel[ty][b][a * D + l];
            for (int k = 0; k < D; ++k) t.Sdiv[k][o] += t.Bel[ty][a][b * D + k];
            t.Sc[o] += t.Cel[ty][a][b];
        }
    }
    // the bulk kernels rely on the decoupled structure of isoviscous rows:
    // a_tr rows equal Laplacian rows (eq. equivalence-stencil), no coupling
    // between components, no weight on the diagonal directions, and the
    // same for C.
    for (int l = 0; l < D; ++l)
        for (int k = 0; k < D; ++k)
            for (int o = 0; o < NB; ++o) {
                const double lap = t.Svis[0][l][k][o], tr = t.Svis[2][l][k][o];
                if (std::fabs(lap - tr) > 1e-13) return fail(ISS_E_INVAL, "a_tr bulk stencil != Laplacian");
                if ((k != l || o > 2 * D) && std::fabs(lap) > 1e-13)
                    return fail(ISS_E_INVAL, "Laplacian stencil not decoupled / axis-only");
                t.Svis[2][l][k][o] = lap;   // identical by construction
            }
    for (int o = 2 * D + 1; o < NB; ++o)
        if (std::fabs(t.Sc[o]) > 1e-13) return fail(ISS_E_INVAL, "C stencil not axis-only");
    // the right-hand-side kernels use the compile-time integer stencils
    const double vol = kuhn_volume<D>(), bvol = -vol / (D + 1);
    for (int o = 0; o < NB; ++o) {
        for (int f = 0; f < 3; ++f)
            for (int l = 0; l < D; ++l)
                for (int k = 0; k < D; ++k)
                    if (std::fabs(t.Svis[f][l][k][o] - vol * svis_int<D>(f, l, k, o)) > 1e-13)
                        return fail(ISS_E_INVAL, "viscous stencil (integer form)");
        if (std::fabs(t.Sc[o] - vol * sc_int<D>(o)) > 1e-13) return fail(ISS_E_INVAL, "C stencil (integer form)");
        for (int k = 0; k < D; ++k) {
            if (std::fabs(t.Sdiv[k][o] - bvol * sdiv_int<D>(k, o)) > 1e-13)
                return fail(ISS_E_INVAL, "B stencil (integer form)");
            if (std::fabs(t.Sbt[k][o] - bvol * sbt_int<D>(k, o)) > 1e-13)
                return fail(ISS_E_INVAL, "B^T stencil (integer form)");
        }
    }
    return ISS_OK;
}

template <int D>
void to_float(const ElemTables<D, double>& a, ElemTables<D, float>& b) {
    const double* s = reinterpret_cast<const double*>(&a);
    float* d = reinterpret_cast<float*>(&b);
    const size_t n = sizeof(a) / sizeof(double);
    for (size_t i = 0; i < n; ++i) d[i] = (float)s[i];
}

// ----------------------------------------------------------------------------
// problem data

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Level {
    LevelView v{};
    LevelView v16{};                // the same level for the scaled FP16 V-cycle (S K S)
    uint8_t* d_vphase = nullptr;
    uint8_t* d_vphase_s = nullptr;  // phase bytes in the colour-split layout
    int32_t* d_spec = nullptr;
    uint8_t* d_spec_eph = nullptr;
    std::vector<uint8_t> cls;       // per vertex: bit0 interface, bit1 boundary
    std::vector<uint8_t> elem_phase;// per element (cell * NT + type)
    std::vector<double> mu_tab, imu_tab;     // viscosity and 1/viscosity per phase
    std::vector<double> emu, eimu;  // per element averages (setup only)
    std::vector<uint8_t> h_vphase;  // finest level: host copy of the phase bytes
    std::vector<int32_t> h_spec;    // finest level: special vertices
    std::vector<uint8_t> h_eph;     // finest level: their slot phases
    double* d_mu64 = nullptr;
    double* d_imu64 = nullptr;
    float* d_mu32 = nullptr;
    float* d_imu32 = nullptr;
    int64_t ninterface = 0, nboundary = 0;
    // work vectors per storage precision (PREC_F64 .. PREC_F16)
    void* w_x[NPREC] = {};
    void* w_b[NPREC] = {};
    void* w_r[NPREC] = {};
    void* w_s[NPREC] = {};   // split layout: xs, bs, ws (d+1 fields each)
};

struct Coarse {
    int64_t M = 0;                  // free dofs + 1 (border)
    std::vector<int32_t> free_idx;
    int32_t* d_free = nullptr;
    double* d_Kinv[3] = {nullptr, nullptr, nullptr};
    double* d_Kinv_mod[3] = {nullptr, nullptr, nullptr};   // K^-1 T: right-hand side modified
    double* d_bc = nullptr;
    double* d_xc = nullptr;
    // Krylov coarse solver (option coarse_solver = ISS_COARSE_MINRES)
    bool kr_ready = false;
    KrylovBufs kb{};
    double* d_inv_diag[3] = {nullptr, nullptr, nullptr};   // per form
    double* d_bb = nullptr;
    double* d_xx = nullptr;
    int32_t* d_all = nullptr;                               // 0 .. (d+1) N - 1
};

}  // namespace

// the part of a V-cycle below the finest level (for one form of the call on
// the finest level), recorded once as a HIP graph
struct VGraph {
    bool warm = false;              // one eager run done (buffers and coarse inverse exist)
    hipGraphExec_t exec = nullptr;
};

struct iss_problem {
    int dim = 3, macro = 1, levels = 0, coarse = 0;
    std::vector<iss_inclusion> inc;
    std::vector<double> mu;
    iss_options opt{};
    std::vector<Level> lv;          // index = level
    double* d_mu64 = nullptr;
    double* d_imu64 = nullptr;
    float* d_mu32 = nullptr;
    float* d_imu32 = nullptr;
    Coarse cs;
    ElemTables<3, double> t3{};
    ElemTables<2, double> t2{};
    // reductions
    double* d_partial = nullptr;    // 1024 * 64 doubles
    double* d_red = nullptr;        // 64 doubles
    // Krylov workspace (finest level, FP64)
    int kry_m = 0;
    double* d_V = nullptr;
    double* d_Z = nullptr;
    double* d_w = nullptr;
    double* d_r = nullptr;
    double* d_h = nullptr;          // m + 2 entries
    double* d_rate = nullptr;       // asymptotic-rate measurement: b = 0 and K x (2 vectors)
    uint8_t* d_flag = nullptr;      // 256 buoyancy flags
    uint8_t* d_eph = nullptr;       // finest-level element phases (P1-P0 calls)
    double* h_pinned = nullptr;     // 8192 doubles of pinned host memory
    int64_t reorth_count = 0;       // second Gram-Schmidt passes (diagnostics)
    iss_net* net = nullptr;         // attached band correction (not owned)
    std::vector<iss_net*> nets;     // every network created for this problem
    int net_accepted = 0, net_rejected = 0;
    // coarse part of the V-cycle per (form, precision) as a HIP graph;
    // ISS_VCYCLE_GRAPH=0 in the environment at creation turns it off
    bool use_graphs = true;
    VGraph vgraph[3][NPREC];
    hipStream_t cap_stream = nullptr;
    int64_t launch_count[ISS_L_KINDS] = {};   // smoother launches per kernel shape
    // caller-owned workspace (iss_bind_workspace): work vectors, the Krylov
    // arrays and the rate buffers are carved from it instead of hipMalloc
    char* ws_base = nullptr;
    size_t ws_size = 0, ws_used = 0;
    std::vector<uint8_t> elem_in;   // per-element phases given at creation (finest level)
    // scaled FP16 V-cycle: K~ = S K S with S = diag(sig_u on velocity,
    // sig_p on pressure); f16_scaled marks the V-cycles run on K~
    double sig_u = 1.0, sig_p = 1.0;
    bool f16_scaled = false;
    double* d_f16mul = nullptr;     // [gamma sig_f | sig_f / gamma] of the current input
    int nphase = 1;
    int device = 0;                 // HIP device current at creation
    void* scratch_dev = nullptr;    // that device's address of `scratch`
    std::vector<void*> allocs;
};

struct iss_net {
    iss_problem* p = nullptr;
    iss::NetImpl* impl = nullptr;
};

namespace {

// Device address of `scratch` on the current device, resolved once per
// device (each GPU holds its own copy at its own address).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_address(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) return fail(ISS_E_INVAL, "device id out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ISS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ISS_OK;
}

int dev_alloc(iss_problem* p, void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) return fail(ISS_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    p->allocs.push_back(*ptr);
    return ISS_OK;
}

// Work buffers: from the bound workspace if there is one (256-byte
// aligned bump allocation), else hipMalloc.
constexpr size_t WS_ALIGN = 256;
inline size_t ws_round(size_t b) { return (b + WS_ALIGN - 1) & ~(WS_ALIGN - 1); }

int work_alloc(iss_problem* p, void** ptr, size_t bytes) {
    if (!p->ws_base) return dev_alloc(p, ptr, bytes);
    *ptr = nullptr;
    const size_t need = ws_round(std::max<size_t>(bytes, 8));
    if (p->ws_used + need > p->ws_size)
        return fail(ISS_E_NOWS, "workspace too small: " + std::to_string(p->ws_used + need) + " bytes needed, " +
                                    std::to_string(p->ws_size) + " bound");
    *ptr = p->ws_base + p->ws_used;
    p->ws_used += need;
    return ISS_OK;
}

template <typename T>
int dev_upload(iss_problem* p, T** ptr, const T* host, size_t count) {
    int rc = dev_alloc(p, (void**)ptr, count * sizeof(T));
    if (rc) return rc;
    if (count) ISS_HIP(hipMemcpy(*ptr, host, count * sizeof(T), hipMemcpyHostToDevice));
    return ISS_OK;
}

// phase of an element by the centroid rule
int element_phase(const iss_problem* p, const double (&c)[3]) {
    for (const auto& in : p->inc) {
        bool inside;
        if (in.kind == ISS_SPHERE) {
            double r2 = 0;
            for (int a = 0; a < p->dim; ++a) r2 += (c[a] - in.a[a]) * (c[a] - in.a[a]);
            inside = r2 < in.a[3] * in.a[3];
        } else if (in.kind == ISS_HALFSPACE) {
            inside = c[(int)in.a[0]] < in.a[1];
        } else {
            inside = true;
            for (int a = 0; a < p->dim; ++a) inside = inside && c[a] > in.a[2 * a] && c[a] < in.a[2 * a + 1];
        }
        if (inside) return in.phase;
    }
    return 0;
}

// Element phases of level l by the centroid rule with the problem's table.
template <int D>
void centroid_phases(iss_problem* p, int l) {
    constexpr auto& K = Kuhn<D>::T;
    constexpr int NT = KuhnTables<D>::NT;
    Level& L = p->lv[l];
    const int n = p->macro << l;
    const int64_t ncell = (D == 3) ? (int64_t)n * n * n : (int64_t)n * n;
    L.elem_phase.assign(ncell * NT, 0);
    const bool given = l == p->levels && !p->elem_in.empty();
    if (given) {
        L.elem_phase = p->elem_in;                // phases given per element
        std::vector<uint8_t>().swap(p->elem_in);
    }
#pragma omp parallel for schedule(static) if (!given)
    for (int64_t c = 0; c < (given ? 0 : ncell); ++c) {
        const int ci = (int)(c % n), cj = (int)((c / n) % n), ck = (D == 3) ? (int)(c / ((int64_t)n * n)) : 0;
        for (int ty = 0; ty < NT; ++ty) {
            double cen[3] = {0, 0, 0};
            for (int b = 0; b <= D; ++b) {
                cen[0] += ci + K.type_vert[ty][b][0];
                cen[1] += cj + K.type_vert[ty][b][1];
                cen[2] += ck + K.type_vert[ty][b][2];
            }
            for (int a = 0; a < 3; ++a) cen[a] /= (double)(D + 1) * n;
            L.elem_phase[c * NT + ty] = (uint8_t)element_phase(p, cen);
        }
    }
    // 256 entries: every phase byte, including the unused ones and the
    // OUTSIDE / SPECIAL marker 255, indexes a defined entry
    L.mu_tab.assign(256, 1.0);
    std::copy(p->mu.begin(), p->mu.end(), L.mu_tab.begin());
    L.imu_tab.resize(256);
    for (int i = 0; i < 256; ++i) L.imu_tab[i] = 1.0 / L.mu_tab[i];
}

// Kuhn type of the simplex of a unit cell that contains a point with
// fractional coordinates f (strictly inside): the axis order of decreasing
// f is the permutation of the type.
template <int D>
int kuhn_type_of(const double (&f)[3]) {
    constexpr auto& K = Kuhn<D>::T;
    for (int ty = 0; ty < KuhnTables<D>::NT; ++ty) {
        bool ok = true;
        for (int s = 0; s + 1 < D; ++s) {
            int a0 = -1, a1 = -1;
            for (int a = 0; a < D; ++a) {
                if (K.type_vert[ty][s + 1][a] != K.type_vert[ty][s][a]) a0 = a;
                if (K.type_vert[ty][s + 2][a] != K.type_vert[ty][s + 1][a]) a1 = a;
            }
            ok = ok && f[a0] >= f[a1];
        }
        if (ok) return ty;
    }
    return 0;
}

// Element viscosity of level l as the volume average over the nested
// elements of level l+1 (each coarse simplex is the union of its 8 (4 in
// 2D) equal-volume children).  For nested P1 spaces this makes the coarse
// viscous block the Galerkin product P^T A P; 1/viscosity is averaged the
// same way for the stabilisation block.
template <int D>
void averaged_viscosity(iss_problem* p, int l) {
    constexpr auto& K = Kuhn<D>::T;
    constexpr int NT = KuhnTables<D>::NT;
    Level& F = p->lv[l + 1];
    Level& L = p->lv[l];
    const int nf = p->macro << (l + 1), nc = p->macro << l;
    const int64_t ncf = (D == 3) ? (int64_t)nf * nf * nf : (int64_t)nf * nf;
    const int64_t ncc = (D == 3) ? (int64_t)nc * nc * nc : (int64_t)nc * nc;
    if (F.emu.empty()) {       // finest level: from the phases
        F.emu.resize(ncf * NT);
        F.eimu.resize(ncf * NT);
        for (int64_t e = 0; e < ncf * NT; ++e) {
            F.emu[e] = F.mu_tab[F.elem_phase[e]];
            F.eimu[e] = F.imu_tab[F.elem_phase[e]];
        }
    }
    L.emu.assign(ncc * NT, 0.0);
    L.eimu.assign(ncc * NT, 0.0);
    const double w = 1.0 / (D == 3 ? 8.0 : 4.0);
    for (int64_t c = 0; c < ncf; ++c) {
        const int ci = (int)(c % nf), cj = (int)((c / nf) % nf), ck = (D == 3) ? (int)(c / ((int64_t)nf * nf)) : 0;
        const int cf[3] = {ci, cj, ck};
        for (int ty = 0; ty < NT; ++ty) {
            double cen[3] = {0, 0, 0};
            for (int b = 0; b <= D; ++b)
                for (int a = 0; a < D; ++a) cen[a] += cf[a] + K.type_vert[ty][b][a];
            int cc[3] = {0, 0, 0};
            double fr[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) {
                const double x = cen[a] / (D + 1) / 2.0;      // coarse lattice units
                cc[a] = std::min((int)std::floor(x), nc - 1);
                fr[a] = x - cc[a];
            }
            const int tyc = kuhn_type_of<D>(fr);
            const int64_t ce = (D == 3) ? cc[0] + (int64_t)nc * (cc[1] + (int64_t)nc * cc[2]) : cc[0] + (int64_t)nc * cc[1];
            L.emu[ce * NT + tyc] += w * F.emu[c * NT + ty];
            L.eimu[ce * NT + tyc] += w * F.eimu[c * NT + ty];
        }
    }
    std::vector<double>().swap(F.emu);
    std::vector<double>().swap(F.eimu);
    // phases: one per distinct pure viscosity of the problem, then one per
    // distinct mixed average when they all fit the 254-entry table, else at
    // most 250 logarithmic bins of the mixed averages (each bin stores the
    // mean of its members; relative width below 4% for contrasts up to 1e4)
    std::vector<double> tab_mu, tab_imu;
    std::vector<double> sum_mu(256, 0.0), sum_imu(256, 0.0), cnt(256, 0.0);
    double lo = 1e300, hi = -1e300;
    const int64_t ne = ncc * NT;
    L.elem_phase.assign(ne, 0);
    std::vector<int> pure_of(p->mu.size(), -1);
    std::vector<double> pure_vals;
    auto pure_index = [&](double m, double im) -> int {
        for (size_t k = 0; k < pure_vals.size(); ++k)
            if (pure_vals[k] == m && std::fabs(im * m - 1.0) < 1e-12) return (int)k;
        return -1;
    };
    for (int64_t e = 0; e < ne; ++e) {
        const double m = L.emu[e], im = L.eimu[e];
        bool pure = false;
        for (size_t k = 0; k < p->mu.size() && k < 254; ++k)
            if (std::fabs(m - p->mu[k]) <= 1e-14 * p->mu[k] && std::fabs(im * p->mu[k] - 1.0) < 1e-12) {
                if (pure_index(p->mu[k], 1.0 / p->mu[k]) < 0) pure_vals.push_back(p->mu[k]);
                pure = true;
                break;
            }
        if (!pure) { lo = std::min(lo, std::log(m)); hi = std::max(hi, std::log(m)); }
    }
    const int npure = (int)pure_vals.size();
    // the distinct mixed averages, kept exactly when they fit the table
    std::vector<std::pair<double, double>> mixed;
    for (int64_t e = 0; e < ne; ++e) {
        const double m = L.emu[e], im = L.eimu[e];
        bool pure = false;
        for (int q = 0; q < npure && !pure; ++q)
            pure = std::fabs(m - pure_vals[q]) <= 1e-14 * pure_vals[q] && std::fabs(im * pure_vals[q] - 1.0) < 1e-12;
        if (!pure) mixed.emplace_back(m, im);
    }
    std::sort(mixed.begin(), mixed.end());
    mixed.erase(std::unique(mixed.begin(), mixed.end()), mixed.end());
    const bool exact = npure + (int64_t)mixed.size() <= 254;
    const int nbins = exact ? (int)mixed.size() : std::max(1, std::min(250, 254 - npure));
    std::vector<int> bin_of_elem(ne, -1);
    for (int64_t e = 0; e < ne; ++e) {
        const double m = L.emu[e], im = L.eimu[e];
        int k = -1;
        for (int q = 0; q < npure; ++q)
            if (std::fabs(m - pure_vals[q]) <= 1e-14 * pure_vals[q] && std::fabs(im * pure_vals[q] - 1.0) < 1e-12) k = q;
        if (k < 0 && exact) {
            k = npure + (int)(std::lower_bound(mixed.begin(), mixed.end(), std::make_pair(m, im)) - mixed.begin());
        } else if (k < 0) {
            const double t = (hi > lo) ? (std::log(m) - lo) / (hi - lo) : 0.0;
            k = npure + std::min(nbins - 1, (int)(t * nbins));
        }
        bin_of_elem[e] = k;
        sum_mu[k] += m;
        sum_imu[k] += im;
        cnt[k] += 1;
    }
    std::vector<int> remap(256, -1);
    L.mu_tab.assign(256, 1.0);
    L.imu_tab.assign(256, 1.0);
    int nph = 0;
    for (int k = 0; k < npure + nbins; ++k) {
        if (cnt[k] == 0) continue;
        remap[k] = nph;
        if (k < npure) {
            L.mu_tab[nph] = pure_vals[k];
            L.imu_tab[nph] = 1.0 / pure_vals[k];
        } else if (exact) {
            L.mu_tab[nph] = mixed[k - npure].first;
            L.imu_tab[nph] = mixed[k - npure].second;
        } else {
            L.mu_tab[nph] = sum_mu[k] / cnt[k];
            L.imu_tab[nph] = sum_imu[k] / cnt[k];
        }
        ++nph;
    }
    for (int64_t e = 0; e < ne; ++e) L.elem_phase[e] = (uint8_t)remap[bin_of_elem[e]];
    if (l == p->coarse) { std::vector<double>().swap(L.emu); std::vector<double>().swap(L.eimu); }
}

// Run length q of the colour-split layout: ceil(n1 / M), rounded up to a
// multiple of 16 entries (FP64 runs and rows start on 128-byte L2 lines) or
// else of 8 (64-byte sectors) where that adds at most a quarter.  Aligned
// runs keep a colour phase's reads and its run writes off lines shared with
// other runs: the FP64 velocity colour phase at 257^3 (q 65 -> 80) takes
// 95 instead of 109 us.  Small levels keep q unpadded.  align > 0 (option
// split_align) forces a multiple of align instead.
int split_run_length(int64_t n1, int M, int align) {
    const int64_t q = (n1 + M - 1) / M;
    if (align > 0) return (int)((q + align - 1) / align * align);
    for (int pad : {16, 8}) {
        const int64_t qp = (q + pad - 1) / pad * pad;
        if (4 * qp <= 5 * q) return (int)qp;
    }
    return (int)q;
}

template <int D>
int setup_level(iss_problem* p, int l) {
    constexpr auto& K = Kuhn<D>::T;
    constexpr int NT = KuhnTables<D>::NT, NS = KuhnTables<D>::NS;
    Level& L = p->lv[l];
    const int n = p->macro << l;
    const int64_t n1 = n + 1;
    const int64_t N = (D == 3) ? n1 * n1 * n1 : n1 * n1;
    // vertex classes
    std::vector<uint8_t> vphase(N);
    L.cls.assign(N, 0);
    std::vector<uint8_t> slotph((size_t)N * 0);   // built only for special vertices below
    std::vector<std::vector<int32_t>> spec_by_col(2 * (D + 1));   // [colour] boundary, [D+1+colour] interior
    std::vector<std::vector<uint8_t>> eph_by_col(2 * (D + 1));
    int64_t nif = 0, nbd = 0;
    const int nthr = 1;
    (void)nthr;
    for (int64_t v = 0; v < N; ++v) {
        const int i = (int)(v % n1), j = (int)((v / n1) % n1), k = (D == 3) ? (int)(v / (n1 * n1)) : 0;
        const int ijk[3] = {i, j, k};
        bool bnd = false;
        for (int a = 0; a < D; ++a) bnd = bnd || ijk[a] == 0 || ijk[a] == n;
        uint8_t ph[NS];
        int first = -1;
        bool mixed_phase = false, mixed_mu = false;
        for (int s = 0; s < NS; ++s) {
            int cc[3];
            bool in = true;
            for (int a = 0; a < D; ++a) {
                cc[a] = ijk[a] + K.slot_cell[s][a];
                in = in && cc[a] >= 0 && cc[a] < n;
            }
            if (!in) { ph[s] = OUTSIDE; continue; }
            const int64_t cell = (D == 3) ? cc[0] + (int64_t)n * (cc[1] + (int64_t)n * cc[2]) : cc[0] + (int64_t)n * cc[1];
            ph[s] = L.elem_phase[cell * NT + K.slot_type[s]];
            if (first < 0) first = ph[s];
            else {
                if (ph[s] != first) mixed_phase = true;
                if (L.mu_tab[ph[s]] != L.mu_tab[first]) mixed_mu = true;
            }
        }
        if (mixed_mu) { L.cls[v] |= 1; ++nif; }
        if (bnd) { L.cls[v] |= 2; ++nbd; }
        if (bnd || mixed_phase) {
            vphase[v] = SPECIAL;
            // per colour: boundary vertices first, then interior ones, so
            // that waves of the special kernels mostly take one path
            const int col = (i + j + k) % (D + 1) + (bnd ? 0 : D + 1);
            spec_by_col[col].push_back((int32_t)v);
            eph_by_col[col].insert(eph_by_col[col].end(), ph, ph + NS);
        } else {
            vphase[v] = (uint8_t)first;
        }
    }
    L.ninterface = nif;
    L.nboundary = nbd;
    std::vector<int32_t> spec;
    std::vector<uint8_t> eph;
    int64_t off[5] = {0, 0, 0, 0, 0};
    for (int c = 0; c <= D; ++c) {
        off[c] = (int64_t)spec.size();
        for (int part : {c, D + 1 + c}) {
            spec.insert(spec.end(), spec_by_col[part].begin(), spec_by_col[part].end());
            eph.insert(eph.end(), eph_by_col[part].begin(), eph_by_col[part].end());
        }
    }
    for (int c = D + 1; c < 5; ++c) off[c] = (int64_t)spec.size();
    int64_t mid[4] = {0, 0, 0, 0};
    for (int c = 0; c <= D; ++c) mid[c] = off[c] + (int64_t)spec_by_col[c].size();
    if (l == p->levels) {
        L.h_vphase = vphase;
        L.h_spec = spec;
        L.h_eph = eph;
    }
    int rc;
    {
        std::vector<float> m32(256), im32(256);
        for (int i = 0; i < 256; ++i) { m32[i] = (float)L.mu_tab[i]; im32[i] = (float)L.imu_tab[i]; }
        if ((rc = dev_upload(p, &L.d_mu64, L.mu_tab.data(), 256))) return rc;
        if ((rc = dev_upload(p, &L.d_imu64, L.imu_tab.data(), 256))) return rc;
        if ((rc = dev_upload(p, &L.d_mu32, m32.data(), 256))) return rc;
        if ((rc = dev_upload(p, &L.d_imu32, im32.data(), 256))) return rc;
    }
    if ((rc = dev_upload(p, &L.d_vphase, vphase.data(), vphase.size()))) return rc;
    // colour-split layout of the smoother: rows grouped by i mod (d+1)
    constexpr int M = D + 1;
    const int q = split_run_length(n1, M, p->opt.split_align);
    const int64_t Rp = (int64_t)M * q;
    const int64_t Pp = Rp * n1;
    const int64_t Ns = (D == 3) ? Pp * n1 : Rp * n1;
    {
        std::vector<uint8_t> vs((size_t)Ns, SPECIAL);
        for (int64_t v = 0; v < N; ++v) {
            const int64_t row = v / n1;
            const int i = (int)(v - row * n1);
            vs[(size_t)(row * Rp + (int64_t)(i % M) * q + i / M)] = vphase[v];
        }
        if ((rc = dev_upload(p, &L.d_vphase_s, vs.data(), vs.size()))) return rc;
    }
    if ((rc = dev_upload(p, &L.d_spec, spec.data(), spec.size()))) return rc;
    if ((rc = dev_upload(p, &L.d_spec_eph, eph.data(), eph.size()))) return rc;
    LevelView& V = L.v;
    V.dim = D;
    V.n = n;
    V.N = N;
    V.sy = n1;
    V.sz = (D == 3) ? n1 * n1 : 0;
    V.vphase = L.d_vphase;
    V.spec = L.d_spec;
    V.spec_eph = L.d_spec_eph;
    for (int c = 0; c < 5; ++c) V.spec_off[c] = off[c];
    for (int c = 0; c < 4; ++c) V.spec_mid[c] = mid[c];
    V.mu64 = L.d_mu64;
    V.imu64 = L.d_imu64;
    V.mu32 = L.d_mu32;
    V.imu32 = L.d_imu32;
    const double h = 1.0 / n;
    V.sA = std::pow(h, D - 2);
    V.sB = std::pow(h, D - 1);
    V.sC = p->opt.stab_beta * std::pow(h, D);
    V.q = q;
    V.Rp = (int)Rp;
    V.Pp = Pp;
    V.Ns = Ns;
    V.vphase_s = L.d_vphase_s;
    V.merge_max_n = p->opt.merge_max_n;
    V.spec_wide_min = p->opt.spec_wide_min;
    V.launch_count = p->launch_count;
    V.freeslip = p->opt.bc == ISS_BC_FREESLIP;
    return ISS_OK;
}

int ensure_work(iss_problem* p, int l, int prec) {
    Level& L = p->lv[l];
    if (L.w_x[prec]) return ISS_OK;
    const size_t bytes = (size_t)(p->dim + 1) * L.v.N * prec_bytes(prec);
    int rc;
    if ((rc = work_alloc(p, &L.w_x[prec], bytes))) return rc;
    if ((rc = work_alloc(p, &L.w_b[prec], bytes))) return rc;
    if ((rc = work_alloc(p, &L.w_r[prec], bytes))) return rc;
    const size_t sbytes = (size_t)3 * (p->dim + 1) * L.v.Ns * prec_bytes(prec);
    if ((rc = work_alloc(p, &L.w_s[prec], sbytes))) return rc;
    return ISS_OK;
}

// split-layout buffers of a level: xs, bs, ws (d+1 fields of Ns each)
void split_buffers(iss_problem* p, int l, int prec, void** xs, void** bs, void** ws) {
    const Level& L = p->lv[l];
    const size_t vec = (size_t)(p->dim + 1) * L.v.Ns * prec_bytes(prec);
    char* base = (char*)L.w_s[prec];
    *xs = base;
    *bs = base + vec;
    *ws = base + 2 * vec;
}

// ----------------------------------------------------------------------------
// velocity component f of vertex v (lattice of n cells per axis) is fixed:
// every component on the boundary for no-slip, the normal one on each face
// for free-slip (eq. boundary)
bool velocity_fixed(const iss_problem* p, int n, int64_t v, int f) {
    const int64_t n1 = n + 1;
    int ijk[3] = {(int)(v % n1), (int)((v / n1) % n1), p->dim == 3 ? (int)(v / (n1 * n1)) : 0};
    if (p->opt.bc == ISS_BC_FREESLIP) return ijk[f] == 0 || ijk[f] == n;
    for (int a = 0; a < p->dim; ++a)
        if (ijk[a] == 0 || ijk[a] == n) return true;
    return false;
}

// coarse level: dense bordered matrix, LU with partial pivoting, inverse

template <int D>
void coarse_matrix(const iss_problem* p, int form, std::vector<double>& Kd, int64_t& M,
                   std::vector<int32_t>& free_idx) {
    constexpr auto& K = Kuhn<D>::T;
    constexpr int NT = KuhnTables<D>::NT;
    const ElemTables<D, double>& E = *reinterpret_cast<const ElemTables<D, double>*>(
        D == 3 ? (const void*)&p->t3 : (const void*)&p->t2);
    const Level& L = p->lv[p->coarse];
    const int n = L.v.n;
    const int64_t n1 = n + 1, N = L.v.N;
    // compact numbering of free dofs: the velocity components that are not
    // fixed by the boundary condition, every pressure
    std::vector<int64_t> cmap((size_t)(D + 1) * N, -1);
    free_idx.clear();
    for (int f = 0; f <= D; ++f)
        for (int64_t v = 0; v < N; ++v)
            if (f == D || !velocity_fixed(p, n, v, f)) {
                cmap[(size_t)f * N + v] = (int64_t)free_idx.size();
                free_idx.push_back((int32_t)((int64_t)f * N + v));
            }
    const int64_t m = (int64_t)free_idx.size();
    M = m + 1;
    Kd.assign((size_t)M * M, 0.0);
    const double sA = L.v.sA, sB = L.v.sB, sC = L.v.sC;
    std::vector<double> w(N, 0.0);
    const int64_t ncell = (D == 3) ? (int64_t)n * n * n : (int64_t)n * n;
    for (int64_t c = 0; c < ncell; ++c) {
        const int ci = (int)(c % n), cj = (int)((c / n) % n), ck = (D == 3) ? (int)(c / ((int64_t)n * n)) : 0;
        for (int ty = 0; ty < NT; ++ty) {
            const int ph = L.elem_phase[c * NT + ty];
            const double mu = L.mu_tab[ph], imu = L.imu_tab[ph];
            int64_t vid[D + 1];
            for (int b = 0; b <= D; ++b)
                vid[b] = (ci + K.type_vert[ty][b][0]) + n1 * (cj + K.type_vert[ty][b][1]) +
                         (D == 3 ? n1 * n1 * (ck + K.type_vert[ty][b][2]) : 0);
            double vol = 1.0;
            for (int a = 0; a < D; ++a) vol /= n;
            vol /= (D == 3 ? 6.0 : 2.0);
            for (int a = 0; a <= D; ++a) {
                w[vid[a]] += vol * imu / (D + 1);
                for (int b = 0; b <= D; ++b) {
                    // velocity-velocity and B^T / B couplings
                    for (int l = 0; l < D; ++l) {
                        const int64_t r = cmap[(size_t)l * N + vid[a]];
                        if (r < 0) continue;
                        for (int k = 0; k < D; ++k) {
                            const int64_t cc = cmap[(size_t)k * N + vid[b]];
                            if (cc >= 0) Kd[(size_t)r * M + cc] += mu * sA * E.Avis[form][ty][a * D + l][b * D + k];
                        }
                        const int64_t cp = cmap[(size_t)D * N + vid[b]];
                        Kd[(size_t)r * M + cp] += sB * E.Bel[ty][b][a * D + l];
                    }
                    const int64_t rp = cmap[(size_t)D * N + vid[a]];
                    for (int k = 0; k < D; ++k) {
                        const int64_t cc = cmap[(size_t)k * N + vid[b]];
                        if (cc >= 0) Kd[(size_t)rp * M + cc] += sB * E.Bel[ty][a][b * D + k];
                    }
                    Kd[(size_t)rp * M + cmap[(size_t)D * N + vid[b]]] -= sC * imu * E.Cel[ty][a][b];
                }
            }
        }
    }
    for (int64_t v = 0; v < N; ++v) {
        const int64_t cp = cmap[(size_t)D * N + v];
        Kd[(size_t)cp * M + m] = w[v];
        Kd[(size_t)m * M + cp] = w[v];
    }
}

// In-place inverse of a dense M x M matrix (row major) by LU with partial
// pivoting followed by column-wise triangular solves.
int dense_inverse(std::vector<double>& A, int64_t M) {
    std::vector<int64_t> piv(M);
    for (int64_t c = 0; c < M; ++c) {
        int64_t pr = c;
        double best = std::fabs(A[(size_t)c * M + c]);
        for (int64_t r = c + 1; r < M; ++r) {
            const double v = std::fabs(A[(size_t)r * M + c]);
            if (v > best) { best = v; pr = r; }
        }
        if (best == 0.0) return fail(ISS_E_INVAL, "coarse matrix is singular");
        piv[c] = pr;
        if (pr != c)
            for (int64_t j = 0; j < M; ++j) std::swap(A[(size_t)c * M + j], A[(size_t)pr * M + j]);
        const double d = A[(size_t)c * M + c];
        const double* rowc = &A[(size_t)c * M];
#pragma omp parallel for schedule(static)
        for (int64_t r = c + 1; r < M; ++r) {
            double* rowr = &A[(size_t)r * M];
            const double f = rowr[c] / d;
            rowr[c] = f;
            for (int64_t j = c + 1; j < M; ++j) rowr[j] -= f * rowc[j];
        }
    }
    // solve L U X = P I column by column
    std::vector<double> Inv((size_t)M * M);
#pragma omp parallel
    {
        std::vector<double> col(M);
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < M; ++j) {
            std::fill(col.begin(), col.end(), 0.0);
            col[j] = 1.0;
            for (int64_t c = 0; c < M; ++c)
                if (piv[c] != c) std::swap(col[c], col[piv[c]]);
            for (int64_t r = 0; r < M; ++r) {
                double s = col[r];
                const double* a = &A[(size_t)r * M];
                for (int64_t c = 0; c < r; ++c) s -= a[c] * col[c];
                col[r] = s;
            }
            for (int64_t r = M - 1; r >= 0; --r) {
                double s = col[r];
                const double* a = &A[(size_t)r * M];
                for (int64_t c = r + 1; c < M; ++c) s -= a[c] * col[c];
                col[r] = s / a[r];
            }
            for (int64_t r = 0; r < M; ++r) Inv[(size_t)r * M + j] = col[r];
        }
    }
    A.swap(Inv);
    return ISS_OK;
}

// Preconditioner diagonals of the coarse Krylov solver for `form`: the
// inverse diagonal of the velocity block A (0 on fixed dofs) and the
// inverse lumped pressure mass 1 / w_j, w_j = sum_T |T| / ((d+1) mu_T).
template <int D>
void coarse_jacobi(const iss_problem* p, int form, std::vector<double>& inv_d) {
    constexpr auto& K = Kuhn<D>::T;
    constexpr int NT = KuhnTables<D>::NT;
    const ElemTables<D, double>& E = *reinterpret_cast<const ElemTables<D, double>*>(
        D == 3 ? (const void*)&p->t3 : (const void*)&p->t2);
    const Level& L = p->lv[p->coarse];
    const int n = L.v.n;
    const int64_t n1 = n + 1, N = L.v.N;
    std::vector<double> dg((size_t)(D + 1) * N, 0.0);
    const int64_t ncell = (D == 3) ? (int64_t)n * n * n : (int64_t)n * n;
    double vol = 1.0;
    for (int a = 0; a < D; ++a) vol /= n;
    vol /= (D == 3 ? 6.0 : 2.0);
    for (int64_t c = 0; c < ncell; ++c) {
        const int ci = (int)(c % n), cj = (int)((c / n) % n), ck = (D == 3) ? (int)(c / ((int64_t)n * n)) : 0;
        for (int ty = 0; ty < NT; ++ty) {
            const int ph = L.elem_phase[c * NT + ty];
            const double mu = L.mu_tab[ph], imu = L.imu_tab[ph];
            for (int a = 0; a <= D; ++a) {
                const int64_t v = (ci + K.type_vert[ty][a][0]) + n1 * (cj + K.type_vert[ty][a][1]) +
                                  (D == 3 ? n1 * n1 * (ck + K.type_vert[ty][a][2]) : 0);
                for (int l = 0; l < D; ++l)
                    dg[(size_t)l * N + v] += mu * L.v.sA * E.Avis[form][ty][a * D + l][a * D + l];
                dg[(size_t)D * N + v] += vol * imu / (D + 1);
            }
        }
    }
    inv_d.assign(dg.size(), 0.0);
    for (int64_t v = 0; v < N; ++v) {
        for (int l = 0; l < D; ++l)
            if (!velocity_fixed(p, n, v, l)) inv_d[(size_t)l * N + v] = 1.0 / dg[(size_t)l * N + v];
        inv_d[(size_t)D * N + v] = 1.0 / dg[(size_t)D * N + v];
    }
}

int ensure_minres(iss_problem* p, int form) {
    Coarse& cs = p->cs;
    const Level& L = p->lv[p->coarse];
    const int64_t n = (int64_t)(p->dim + 1) * L.v.N;
    int rc;
    if (!cs.kr_ready) {
        const size_t bytes = (size_t)n * sizeof(double);
        double** vecs[] = {&cs.kb.v[0], &cs.kb.v[1], &cs.kb.v[2], &cs.kb.z[0], &cs.kb.z[1], &cs.kb.w[0],
                           &cs.kb.w[1], &cs.kb.w[2], &cs.kb.q, &cs.kb.t, &cs.kb.u, &cs.kb.r, &cs.kb.zc,
                           &cs.kb.pc, &cs.kb.qc, &cs.d_bb, &cs.d_xx};
        for (double** v : vecs) {
            if ((rc = dev_alloc(p, (void**)v, bytes))) return rc;
            ISS_HIP(hipMemset(*v, 0, bytes));
        }
        if ((rc = dev_alloc(p, (void**)&cs.kb.st, 16 * sizeof(double)))) return rc;
        ISS_HIP(hipMemset(cs.kb.st, 0, 16 * sizeof(double)));
        std::vector<int32_t> all((size_t)n);
        for (int64_t i = 0; i < n; ++i) all[(size_t)i] = (int32_t)i;
        if ((rc = dev_upload(p, &cs.d_all, all.data(), all.size()))) return rc;
        cs.kr_ready = true;
    }
    if (!cs.d_inv_diag[form]) {
        std::vector<double> inv_d;
        if (p->dim == 3) coarse_jacobi<3>(p, form, inv_d);
        else coarse_jacobi<2>(p, form, inv_d);
        if ((rc = dev_upload(p, &cs.d_inv_diag[form], inv_d.data(), inv_d.size()))) return rc;
    }
    return ISS_OK;
}

// Inverse of the bordered coarse matrix of `form`; with mod, the inverse
// times T = [[I, B^T M^-1], [0, I]], M the lumped (1/mu)-weighted pressure
// mass (the weights of the pressure constraint): the coarse right-hand side
// r_1 becomes r_1 + B^T M^-1 r_2 (Sec. 5, coarse grid solver; the sign
// follows b(v, q) = -(div v, q)), which makes the strain-form coarse system
// approximate the a_tr system of the finer levels where div u != 0.
int ensure_coarse(iss_problem* p, int form, bool mod = false) {
    if (p->opt.coarse_solver == ISS_COARSE_MINRES) return ensure_minres(p, form);
    Coarse& cs = p->cs;
    if (mod ? cs.d_Kinv_mod[form] : cs.d_Kinv[form]) return ISS_OK;
    std::vector<double> Kd;
    int64_t M;
    std::vector<int32_t> fidx;
    if (p->dim == 3) coarse_matrix<3>(p, form, Kd, M, fidx);
    else coarse_matrix<2>(p, form, Kd, M, fidx);
    // per pressure column c: the entries of B^T M^-1 in the velocity rows
    std::vector<std::vector<std::pair<int64_t, double>>> E;
    if (mod) {
        const int64_t m = M - 1;
        const int64_t NpStart = (int64_t)p->dim * p->lv[p->coarse].v.N;
        E.resize(M);
        for (int64_t c = 0; c < m; ++c) {
            if (fidx[c] < NpStart) continue;                     // pressure columns only
            const double wj = Kd[(size_t)m * M + c];              // border row: the weight
            for (int64_t r = 0; r < m; ++r)
                if (fidx[r] < NpStart && Kd[(size_t)r * M + c] != 0.0)
                    E[c].emplace_back(r, Kd[(size_t)r * M + c] / wj);
        }
    }
    int rc;
    if ((rc = dense_inverse(Kd, M))) return rc;
    if (mod) {
        // (K^-1 T)[:, c] = K^-1[:, c] + sum_r K^-1[:, r] E[r][c] (row-major)
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            double* row = &Kd[(size_t)i * M];
            std::vector<double> add(M, 0.0);
            for (int64_t c = 0; c < M; ++c)
                for (const auto& e : E[c]) add[c] += row[e.first] * e.second;
            for (int64_t c = 0; c < M; ++c) row[c] += add[c];
        }
    }
    if (!cs.d_free) {
        cs.M = M;
        cs.free_idx = fidx;
        if ((rc = dev_upload(p, &cs.d_free, fidx.data(), fidx.size()))) return rc;
        if ((rc = dev_alloc(p, (void**)&cs.d_bc, M * sizeof(double)))) return rc;
        if ((rc = dev_alloc(p, (void**)&cs.d_xc, M * sizeof(double)))) return rc;
        ISS_HIP(hipMemset(cs.d_bc, 0, M * sizeof(double)));
    }
    if ((rc = dev_upload(p, mod ? &cs.d_Kinv_mod[form] : &cs.d_Kinv[form], Kd.data(), Kd.size()))) return rc;
    return ISS_OK;
}

// the coarse right-hand side is modified when the coarsest level swaps to
// another form than the level above it uses (option coarse_rhs_mod)
int level_form(const iss_problem* p, int l, int form);
bool coarse_mod(const iss_problem* p, int form) {
    return p->opt.coarse_rhs_mod && p->levels > p->coarse &&
           level_form(p, p->coarse, form) != level_form(p, p->coarse + 1, form);
}

// ----------------------------------------------------------------------------
// multigrid

int check_form(int form) { return (form >= 0 && form <= 2) ? ISS_OK : fail(ISS_E_INVAL, "bad form"); }
int check_prec(int prec) { return (prec >= 0 && prec < NPREC) ? ISS_OK : fail(ISS_E_INVAL, "bad precision"); }

// the view of level l a V-cycle in precision prec works with: the scaled
// system inside the FP16 preconditioner, else the level itself
const LevelView& view(const iss_problem* p, int l, int prec) {
    return (prec == PREC_F16 && p->f16_scaled) ? p->lv[l].v16 : p->lv[l].v;
}
int check_level(const iss_problem* p, int l) {
    return (l >= p->coarse && l <= p->levels) ? ISS_OK : fail(ISS_E_INVAL, "level out of range");
}

// Viscous form of level l inside a V-cycle called with `form` on the finest
// level: the finest level keeps the call's form, the levels in between take
// mid_form (default: the call's form), the coarsest takes coarse_form
// (default: that of the levels above it).
int level_form(const iss_problem* p, int l, int form) {
    if (l == p->levels) return form;
    const int mid = p->opt.mid_form >= 0 ? p->opt.mid_form : form;
    if (l == p->coarse) return p->opt.coarse_form >= 0 ? p->opt.coarse_form : mid;
    return mid;
}

int coarse_solve(iss_problem* p, int form, int prec, const void* b, void* x, hipStream_t s, bool mod = false) {
    int rc;
    if ((rc = ensure_coarse(p, form, mod))) return rc;
    Coarse& cs = p->cs;
    const Level& L = p->lv[p->coarse];
    const int64_t m = cs.M - 1;
    // on the scaled system S K S: x~ = S^-1 K^-1 S^-1 b~ (field multipliers)
    FieldMul fm{};
    if (prec == PREC_F16 && p->f16_scaled) {
        for (int f = 0; f <= p->dim; ++f) fm.m[f] = 1.0 / (f < p->dim ? p->sig_u : p->sig_p);
        fm.N = L.v.N;
        fm.on = 1;
    }
    if (p->opt.coarse_solver == ISS_COARSE_MINRES) {
        const int64_t n = (int64_t)(p->dim + 1) * L.v.N;
        KrylovBufs kb = cs.kb;
        kb.inv_d = cs.d_inv_diag[form];
        ISS_HIP(k_gather(prec, b, cs.d_all, n, cs.d_bb, s, fm));
        ISS_HIP(minres_coarse(L.v, form, kb, p->opt.minres_iters, p->opt.minres_cg, mod, cs.d_bb, cs.d_xx, s));
        ISS_HIP(k_scatter(prec, cs.d_xx, cs.d_all, n, x, s, fm));
        return ISS_OK;
    }
    ISS_HIP(k_gather(prec, b, cs.d_free, m, cs.d_bc, s, fm));
    ISS_HIP(k_dense_matvec(mod ? cs.d_Kinv_mod[form] : cs.d_Kinv[form], cs.M, cs.d_bc, cs.d_xc, s));
    ISS_HIP(k_fill(prec, x, (int64_t)(p->dim + 1) * L.v.N, 0.0, s));
    ISS_HIP(k_scatter(prec, cs.d_xc, cs.d_free, m, x, s, fm));
    return ISS_OK;
}

// V(nu1, nu2) cycle on level l for a cycle called with `form` on the finest
// level (each level uses level_form).  x_zero: x holds zero on entry (it is
// then not read).  Smoothing runs on colour-split copies of x and b; b is
// packed once for both smoothing phases.
int vcycle(iss_problem* p, int l, int form, int prec, void* x, const void* b, bool x_zero, hipStream_t s);

// The V-cycle below the finest level touches only the library's per-level
// buffers (restricted residual in, correction out), so after one eager run,
// which allocates them and the coarse inverse, it is recorded once per
// (form, precision) as a HIP graph on a capture stream and replayed on the
// caller's stream: one launch instead of about 1500 short ones per cycle.
// The recording holds kernel launches only (buffers are cleared by fill
// kernels).  If recording fails the problem falls back to eager launches.
int coarse_part(iss_problem* p, int l, int form, int prec, hipStream_t s, bool top) {
    Level& Lc = p->lv[l];
    // (the FP16 graph holds the scaled system: FP16 cycles outside the
    // preconditioner run eagerly)
    if (!top || !p->use_graphs || l == p->coarse || (prec == PREC_F16 && !p->f16_scaled))
        return vcycle(p, l, form, prec, Lc.w_x[prec], Lc.w_b[prec], true, s);
    VGraph& G = p->vgraph[form][prec];
    if (!G.exec) {
        if (!G.warm) {
            const int rc = vcycle(p, l, form, prec, Lc.w_x[prec], Lc.w_b[prec], true, s);
            if (rc == ISS_OK) G.warm = true;
            return rc;
        }
        hipError_t e = hipSuccess;
        if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        int rc = ISS_OK;
        hipGraph_t g = nullptr;
        if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            rc = vcycle(p, l, form, prec, Lc.w_x[prec], Lc.w_b[prec], true, p->cap_stream);
            e = hipStreamEndCapture(p->cap_stream, &g);
        }
        if (rc == ISS_OK && e == hipSuccess && g) e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (rc != ISS_OK || e != hipSuccess || !G.exec) {
            G.exec = nullptr;
            p->use_graphs = false;
            (void)hipGetLastError();
            return vcycle(p, l, form, prec, Lc.w_x[prec], Lc.w_b[prec], true, s);
        }
    }
    ISS_HIP(hipGraphLaunch(G.exec, s));
    return ISS_OK;
}

int vcycle(iss_problem* p, int l, int form, int prec, void* x, const void* b, bool x_zero, hipStream_t s) {
    if (l == p->coarse) return coarse_solve(p, level_form(p, l, form), prec, b, x, s, coarse_mod(p, form));
    const int lform = level_form(p, l, form);
    int rc;
    if ((rc = ensure_work(p, l, prec)) || (rc = ensure_work(p, l - 1, prec))) return rc;
    Level& L = p->lv[l];
    Level& Lc = p->lv[l - 1];
    const LevelView& V = view(p, l, prec);
    const LevelView& Vc = view(p, l - 1, prec);
    const int nf = p->dim + 1;
    void *xs, *bs, *ws;
    split_buffers(p, l, prec, &xs, &bs, &ws);
    ISS_HIP(k_split(V, prec, nf, b, bs, SPLIT_PACK, s));
    if (x_zero) ISS_HIP(k_fill(prec, xs, (int64_t)nf * V.Ns, 0.0, s));
    else ISS_HIP(k_split(V, prec, nf, x, xs, SPLIT_PACK, s));
    const int extra = p->opt.nu_inc * (p->levels - l);      // V_var: more steps on coarser levels
    const int nu1 = p->opt.nu1 + extra, nu2 = p->opt.nu2 + extra;
    for (int i = 0; i < nu1; ++i)
        ISS_HIP(k_smooth_step(V, lform, prec, p->opt.omega, xs, bs, ws, i == 0, s));
    ISS_HIP(k_split(V, prec, nf, xs, x, SPLIT_UNPACK, s));
    ISS_HIP(k_apply(V, lform, BLOCK_FULL, MODE_RESID, prec, x, b, L.w_r[prec], s));
    ISS_HIP(k_restrict(V, Vc, prec, L.w_r[prec], Lc.w_b[prec], s));
    if ((rc = coarse_part(p, l - 1, form, prec, s, l == p->levels))) return rc;
    ISS_HIP(k_prolong_add(V, Vc, prec, Lc.w_x[prec], x, s));
    if (nu2 > 0) {
        ISS_HIP(k_split(V, prec, nf, x, xs, SPLIT_PACK, s));
        for (int i = 0; i < nu2; ++i)
            ISS_HIP(k_smooth_step(V, lform, prec, p->opt.omega, xs, bs, ws, i == 0, s));
        ISS_HIP(k_split(V, prec, nf, xs, x, SPLIT_UNPACK, s));
    }
    return ISS_OK;
}

int field_norms(iss_problem* p, int prec, const void* x, int64_t N, int nf, double* out, hipStream_t s) {
    ISS_HIP(k_field_sumsq(prec, x, N, nf, p->d_partial, p->d_red, s));
    ISS_HIP(hipMemcpyAsync(p->h_pinned, p->d_red, nf * sizeof(double), hipMemcpyDeviceToHost, s));
    ISS_HIP(hipStreamSynchronize(s));
    for (int f = 0; f < nf; ++f) out[f] = p->h_pinned[f];
    return ISS_OK;
}

double total_norm(const double* sq, int nf) {
    double t = 0;
    for (int f = 0; f < nf; ++f) t += sq[f];
    return std::sqrt(t);
}

// z = M^{-1} v: one V-cycle from zero in precision prec (FP64 in, FP64 out)
int precondition(iss_problem* p, int form, int prec, const double* v, double* z, hipStream_t s) {
    const int l = p->levels;
    const int64_t n = (int64_t)(p->dim + 1) * p->lv[l].v.N;
    int rc;
    if ((rc = ensure_work(p, l, prec))) return rc;
    Level& L = p->lv[l];
    if (prec == PREC_F64) {
        for (int c = 0; c < p->opt.cycles; ++c)
            if ((rc = vcycle(p, l, form, PREC_F64, z, v, c == 0, s))) return rc;
    } else if (prec == PREC_F16) {
        // FP16 storage: FP16 holds 5 exponent bits, so the cycle runs on the
        // symmetrically scaled system (S K S) x~ = gamma S v with S the
        // per-field scales of the unit diagonal and gamma the inverse RMS of
        // S v (both on the device), and z = S x~ / gamma.  The cycles are
        // linear, so this is the same preconditioner up to rounding.
        const int nf = p->dim + 1;
        ISS_HIP(k_field_sumsq(PREC_F64, v, L.v.N, nf, p->d_partial, p->d_red, s));
        ISS_HIP(k_f16_multipliers(p->d_red, nf, n, p->sig_u, p->sig_p, p->opt.f16_rms, p->d_f16mul, s));
        ISS_HIP(k_scale_convert(prec, 0, v, L.w_b[prec], L.v.N, nf, p->d_f16mul, s));
        p->f16_scaled = true;
        for (int c = 0; c < p->opt.cycles && rc == ISS_OK; ++c)
            rc = vcycle(p, l, form, prec, L.w_x[prec], L.w_b[prec], c == 0, s);
        p->f16_scaled = false;
        if (rc) return rc;
        ISS_HIP(k_scale_convert(prec, 1, L.w_x[prec], z, L.v.N, nf, p->d_f16mul + nf, s));
    } else {
        // FP32 arithmetic, vectors stored in FP32 or BF16 (same exponent
        // range as FP64 needs here, so no scaling)
        ISS_HIP(k_convert(PREC_F64, v, prec, L.w_b[prec], n, s));
        for (int c = 0; c < p->opt.cycles; ++c)
            if ((rc = vcycle(p, l, form, prec, L.w_x[prec], L.w_b[prec], c == 0, s))) return rc;
        ISS_HIP(k_convert(prec, L.w_x[prec], PREC_F64, z, n, s));
    }
    if (p->net) {
        // band correction of the V-cycle output from the residual it leaves,
        // kept only if it lowers that residual (safeguard)
        iss::NetImpl* nt = p->net->impl;
        double* rp = net_work(nt, 0);
        double* c = net_work(nt, 1);
        double* rpp = net_work(nt, 2);
        ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_RESID, PREC_F64, z, v, rp, s));
        ISS_HIP(net_correction(nt, rp, c, n, s));
        ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_RESID, PREC_F64, c, rp, rpp, s));
        double a[4], b2[4];
        if ((rc = field_norms(p, PREC_F64, rp, L.v.N, p->dim + 1, a, s))) return rc;
        if ((rc = field_norms(p, PREC_F64, rpp, L.v.N, p->dim + 1, b2, s))) return rc;
        const double n0 = total_norm(a, p->dim + 1), n1 = total_norm(b2, p->dim + 1);
        if (std::isfinite(n1) && n1 < n0) {
            ISS_HIP(k_axpby(z, 1.0, c, 1.0, n, s));
            ++p->net_accepted;
        } else {
            ++p->net_rejected;
        }
    }
    return ISS_OK;
}

int ensure_krylov(iss_problem* p, int m) {
    if (p->kry_m >= m && p->d_V) return ISS_OK;
    if (2 * m + 4 > 8192) return fail(ISS_E_INVAL, "restart length too large");
    if (p->d_V && p->ws_base) return fail(ISS_E_NOWS, "Krylov arrays of another restart length in a bound workspace");
    if (p->d_V) {
        (void)hipFree(p->d_V); (void)hipFree(p->d_Z); (void)hipFree(p->d_w); (void)hipFree(p->d_r); (void)hipFree(p->d_h);
        auto rm = [&](void* q) { p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), q), p->allocs.end()); };
        rm(p->d_V); rm(p->d_Z); rm(p->d_w); rm(p->d_r); rm(p->d_h);
    }
    const int64_t n = (int64_t)(p->dim + 1) * p->lv[p->levels].v.N;
    int rc;
    if ((rc = work_alloc(p, (void**)&p->d_V, (size_t)(m + 1) * n * 8))) return rc;
    if ((rc = work_alloc(p, (void**)&p->d_Z, (size_t)m * n * 8))) return rc;
    if ((rc = work_alloc(p, (void**)&p->d_w, (size_t)n * 8))) return rc;
    if ((rc = work_alloc(p, (void**)&p->d_r, (size_t)n * 8))) return rc;
    if ((rc = work_alloc(p, (void**)&p->d_h, (size_t)(2 * m + 4) * 8))) return rc;
    p->kry_m = m;
    return ISS_OK;
}

int solve(iss_problem* p, int form, int prec, double rtol, int maxit, double* x, const double* b,
          iss_solve_info* info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    p->net_accepted = p->net_rejected = 0;
    const int l = p->levels;
    Level& L = p->lv[l];
    const int D = p->dim;
    const int64_t N = L.v.N, n = (int64_t)(D + 1) * N;
    const int m = std::max(1, p->opt.restart);
    int rc;
    if ((rc = ensure_krylov(p, m))) return rc;
    if ((rc = ensure_coarse(p, level_form(p, p->coarse, form), coarse_mod(p, form)))) return rc;
    double sq[4];
    if ((rc = field_norms(p, PREC_F64, b, N, D + 1, sq, s))) return rc;
    const double nb = total_norm(sq, D + 1);
    std::vector<double> hist;
    int its = 0;
    double rel = 0;
    if (nb == 0.0) {
        ISS_HIP(k_fill(PREC_F64, x, n, 0.0, s));
        hist.push_back(0.0);
    } else {
        double* r = p->d_r;
        ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_RESID, PREC_F64, x, b, r, s));
        if ((rc = field_norms(p, PREC_F64, r, N, D + 1, sq, s))) return rc;
        double beta = total_norm(sq, D + 1);
        rel = beta / nb;
        hist.push_back(rel);
        const double rel0 = rel;
        auto bad = [&](double v) { return !std::isfinite(v) || v > 1e3 * std::max(rel0, 1e-300); };
        if (p->opt.outer == ISS_OUTER_RICHARDSON) {
            while (rel > rtol && its < maxit) {
                if ((rc = precondition(p, form, prec, r, p->d_w, s))) return rc;
                ISS_HIP(k_axpby(x, 1.0, p->d_w, 1.0, n, s));
                ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_RESID, PREC_F64, x, b, r, s));
                if ((rc = field_norms(p, PREC_F64, r, N, D + 1, sq, s))) return rc;
                rel = total_norm(sq, D + 1) / nb;
                ++its;
                hist.push_back(rel);
                if (bad(rel)) { rc = ISS_E_DIVERGED; break; }
            }
        } else {
            // Right-preconditioned FGMRES(m) (Saad 1993) with classical
            // Gram-Schmidt and delayed reorthogonalisation: the second
            // projection of each new vector is fused with the first
            // projection of the next one, so each iteration reads the basis
            // twice (one dot pass, one update pass) instead of four times.
            // Column j of V holds the projected, not yet reorthogonalised
            // vector u_j (scaled to about unit length) until step j finishes
            // it; z_j = M u_j (FGMRES accepts any z_j, and u_j differs from
            // v_j only by a multiple plus a vector in span(v_0..v_{j-1})).
            // Column j of the Hessenberg matrix is completed at step j + 1,
            // so convergence is seen one V-cycle late.
            std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
            double* V = p->d_V;
            double* Z = p->d_Z;
            double* w = p->d_w;
            double* dh = p->d_h;
            double* hh = p->h_pinned;
            // Givens rotations on column col (complete) and the residual estimate
            auto close_column = [&](int col) {
                for (int i = 0; i < col; ++i) {
                    const double a = H[(size_t)i * m + col], c = H[(size_t)(i + 1) * m + col];
                    H[(size_t)i * m + col] = cs[i] * a + sn[i] * c;
                    H[(size_t)(i + 1) * m + col] = -sn[i] * a + cs[i] * c;
                }
                const double a = H[(size_t)col * m + col], c = H[(size_t)(col + 1) * m + col];
                const double den = std::hypot(a, c);
                cs[col] = den > 0 ? a / den : 1.0;
                sn[col] = den > 0 ? c / den : 0.0;
                H[(size_t)col * m + col] = den;
                H[(size_t)(col + 1) * m + col] = 0.0;
                g[col + 1] = -sn[col] * g[col];
                g[col] = cs[col] * g[col];
                ++its;
                rel = std::fabs(g[col + 1]) / nb;
                hist.push_back(rel);
            };
            while (rel > rtol && its < maxit && rc == ISS_OK) {
                ISS_HIP(k_scale(V, 1.0 / beta, r, n, s));        // u_0 = v_0 = r / beta
                std::fill(H.begin(), H.end(), 0.0);
                std::fill(g.begin(), g.end(), 0.0);
                g[0] = beta;
                double sig = 1.0;        // u_j = (projected vector of column j-1) / sig
                int done = 0;            // finished Hessenberg columns in this cycle
                bool stop = false;
                for (int j = 0; j < m && !stop; ++j) {
                    if ((rc = precondition(p, form, prec, V + (size_t)j * n, Z + (size_t)j * n, s))) return rc;
                    ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_APPLY, PREC_F64, Z + (size_t)j * n, nullptr, w, s));
                    // pass 1: c = V_{<j}^T u_j, d = V_{<j}^T w, u.u, u.w, w.w
                    ISS_HIP(k_dots2(V, n, j, V + (size_t)j * n, w, n, p->d_partial, dh, s));
                    ISS_HIP(hipMemcpyAsync(hh, dh, (2 * j + 3) * sizeof(double), hipMemcpyDeviceToHost, s));
                    ISS_HIP(hipStreamSynchronize(s));
                    const double* c = hh;
                    const double* d = hh + j;
                    const double uu = hh[2 * j], uw = hh[2 * j + 1], ww = hh[2 * j + 2];
                    double cc = 0, cd = 0, dd = 0;
                    for (int i = 0; i < j; ++i) { cc += c[i] * c[i]; cd += c[i] * d[i]; dd += d[i] * d[i]; }
                    const double a2 = uu - cc;
                    if (!std::isfinite(a2) || !std::isfinite(ww)) { rc = ISS_E_DIVERGED; break; }
                    if (j > 0) {
                        // finish column j - 1: A z_{j-1} = ... + sig (V_{<j} c + alpha v_j)
                        const double alpha = a2 > 1e-28 * uu ? std::sqrt(a2) : 0.0;
                        for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] += sig * c[i];
                        H[(size_t)j * m + (j - 1)] = sig * alpha;
                        close_column(j - 1);
                        done = j;
                        if (!std::isfinite(rel)) { rc = ISS_E_DIVERGED; break; }
                        if (rel <= rtol || alpha == 0.0 || its >= maxit) break;   // z_j is not used
                    }
                    const double alpha = std::sqrt(std::max(a2, 0.0));
                    const double e = (uw - cd) / alpha;
                    for (int i = 0; i < j; ++i) H[(size_t)i * m + j] = d[i];
                    H[(size_t)j * m + j] = e;
                    // length of the new projected vector (Pythagoras; only a scale)
                    const double r2 = ww - dd - e * e;
                    double snew = r2 > 1e-24 * ww ? std::sqrt(r2) : 1e-12 * std::sqrt(ww);
                    if (!(snew > 0) || !std::isfinite(snew)) snew = 1.0;
                    // pass 2: v_j = (u_j - V c) / alpha; u_{j+1} = (w - V d - e v_j) / snew
                    ISS_HIP(k_dcgs_update(V, n, j, dh, dh + j, w, 1.0 / alpha, e, 1.0 / snew, n, s));
                    sig = snew;
                    if (j == m - 1) {
                        // restart: finish the last column with one more dot pass
                        ISS_HIP(k_dots2(V, n, m, V + (size_t)m * n, V + (size_t)m * n, n, p->d_partial, dh, s));
                        ISS_HIP(hipMemcpyAsync(hh, dh, (2 * m + 3) * sizeof(double), hipMemcpyDeviceToHost, s));
                        ISS_HIP(hipStreamSynchronize(s));
                        double c2 = 0;
                        for (int i = 0; i < m; ++i) c2 += hh[i] * hh[i];
                        const double b2 = hh[2 * m] - c2;
                        for (int i = 0; i < m; ++i) H[(size_t)i * m + (m - 1)] += sig * hh[i];
                        H[(size_t)m * m + (m - 1)] = sig * (b2 > 1e-28 * hh[2 * m] ? std::sqrt(b2) : 0.0);
                        close_column(m - 1);
                        done = m;
                        if (!std::isfinite(rel)) { rc = ISS_E_DIVERGED; break; }
                    }
                }
                if (rc != ISS_OK) break;
                const int jn = done;
                if (jn == 0) break;
                // y = H^{-1} g ; x += Z y
                std::vector<double> y(jn);
                for (int i = jn - 1; i >= 0; --i) {
                    double t = g[i];
                    for (int k = i + 1; k < jn; ++k) t -= H[(size_t)i * m + k] * y[k];
                    y[i] = t / H[(size_t)i * m + i];
                }
                std::copy(y.begin(), y.end(), p->h_pinned);
                ISS_HIP(hipMemcpyAsync(dh, p->h_pinned, jn * sizeof(double), hipMemcpyHostToDevice, s));
                ISS_HIP(k_multiaxpy(x, Z, n, jn, dh, 1.0, n, s));
                ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_RESID, PREC_F64, x, b, r, s));
                if ((rc = field_norms(p, PREC_F64, r, N, D + 1, sq, s))) return rc;
                beta = total_norm(sq, D + 1);
                rel = beta / nb;
                hist.back() = rel;
                if (bad(rel)) { rc = ISS_E_DIVERGED; break; }
            }
        }
    }
    ISS_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
        info->net_accepted = p->net_accepted;
        info->net_rejected = p->net_rejected;
        info->iterations = its;
        info->relres = rel;
        info->seconds = secs;
        const int cap = maxit + 1;
        const int cnt = std::min<int>((int)hist.size(), cap);
        info->history_len = info->history ? cnt : 0;
        if (info->history)
            for (int i = 0; i < cnt; ++i) info->history[i] = hist[i];
    }
    if (rc == ISS_E_DIVERGED) return fail(ISS_E_DIVERGED, "solve diverged (residual grew > 1e3 or not finite)");
    if (rc != ISS_OK) return rc;
    if (rel > rtol) return fail(ISS_E_NOTCONV, "maxit reached before tolerance");
    return ISS_OK;
}

}  // namespace

// ============================================================================
// C ABI

extern "C" {

const char* iss_last_error(void) { return g_err.c_str(); }

int iss_default_options(iss_options* o) {
    if (!o) return fail(ISS_E_INVAL, "null options");
    o->nu1 = 3;
    o->nu2 = 3;
    o->omega = 0.3;
    o->stab_beta = 1.0 / 12.0;
    o->outer = ISS_OUTER_RICHARDSON;
    o->restart = 40;
    o->coarse_mu = ISS_COARSE_MU_AVERAGE;
    o->coarse_form = -1;
    o->nu_inc = 0;
    o->mid_form = -1;
    o->merge_max_n = 64;
    o->spec_wide_min = 65536;
    o->cycles = 1;
    o->f16_rms = 1.0 / 1024.0;
    o->coarse_rhs_mod = 0;
    o->bc = ISS_BC_NOSLIP;
    o->split_align = 0;
    o->coarse_solver = ISS_COARSE_DIRECT;
    o->minres_iters = 30;
    o->minres_cg = 5;
    return ISS_OK;
}

void iss_problem_destroy(iss_problem* p) {
    if (!p) return;
    for (iss_net* nt : p->nets) nt->p = nullptr;     // the networks outlive it
    for (auto& row : p->vgraph)
        for (auto& G : row)
            if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (void* q : p->allocs) (void)hipFree(q);
    if (p->h_pinned) (void)hipHostFree(p->h_pinned);
    delete p;
}

static int create_impl(int dim, int macro, int levels, int coarse_level, const iss_inclusion* inclusions,
                       int ninclusions, const uint8_t* elem_phase, const double* mu, int nphase,
                       const iss_options* opt, iss_problem** out);

int iss_problem_create(int dim, int macro, int levels, int coarse_level,
                       const iss_inclusion* inclusions, int ninclusions, const double* mu, int nphase,
                       const iss_options* opt, iss_problem** out) {
    return create_impl(dim, macro, levels, coarse_level, inclusions, ninclusions, nullptr, mu, nphase, opt, out);
}

int iss_problem_create_elems(int dim, int macro, int levels, int coarse_level, const uint8_t* elem_phase,
                             const double* mu, int nphase, const iss_options* opt, iss_problem** out) {
    if (!elem_phase) return fail(ISS_E_INVAL, "null element phases");
    return create_impl(dim, macro, levels, coarse_level, nullptr, 0, elem_phase, mu, nphase, opt, out);
}

static int create_impl(int dim, int macro, int levels, int coarse_level, const iss_inclusion* inclusions,
                       int ninclusions, const uint8_t* elem_phase, const double* mu, int nphase,
                       const iss_options* opt, iss_problem** out) {
    if (!out) return fail(ISS_E_INVAL, "null out");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(ISS_E_INVAL, "dim must be 2 or 3");
    if (macro < 1 || levels < 1 || coarse_level < 1 || coarse_level > levels)
        return fail(ISS_E_INVAL, "need macro >= 1 and 1 <= coarse_level <= levels");
    const int64_t n = (int64_t)macro << levels;
    const int64_t N = (dim == 3) ? (n + 1) * (n + 1) * (n + 1) : (n + 1) * (n + 1);
    if ((int64_t)(dim + 1) * N >= (int64_t)1 << 31) return fail(ISS_E_INVAL, "problem too large for int32 indices");
    {
        // the smoother addresses a split-layout field through 32-bit byte
        // offsets: every FP64 field must stay below 4 GiB
        const int64_t q = split_run_length(n + 1, dim + 1, opt ? opt->split_align : 0);
        const int64_t Ns = (int64_t)(dim + 1) * q * (dim == 3 ? (n + 1) * (n + 1) : (n + 1));
        if (Ns * (int64_t)sizeof(double) >= (int64_t)1 << 32)
            return fail(ISS_E_INVAL, "problem too large: a split-layout field exceeds 4 GiB");
    }
    if (!mu || nphase < 1 || nphase > 254) return fail(ISS_E_INVAL, "need 1 <= nphase <= 254");
    for (int i = 0; i < nphase; ++i)
        if (!(mu[i] > 0) || !std::isfinite(mu[i])) return fail(ISS_E_INVAL, "viscosities must be positive and finite");
    if (ninclusions < 0 || (ninclusions > 0 && !inclusions)) return fail(ISS_E_INVAL, "bad inclusions");
    for (int i = 0; i < ninclusions; ++i) {
        const auto& in = inclusions[i];
        if (in.phase < 0 || in.phase >= nphase) return fail(ISS_E_INVAL, "inclusion phase out of range");
        if (in.kind != ISS_SPHERE && in.kind != ISS_HALFSPACE && in.kind != ISS_BOX)
            return fail(ISS_E_INVAL, "bad inclusion kind");
        if (in.kind == ISS_HALFSPACE && (in.a[0] < 0 || (int)in.a[0] >= dim))
            return fail(ISS_E_INVAL, "half-space axis out of range");
    }
    iss_problem* p = new (std::nothrow) iss_problem();
    if (!p) return fail(ISS_E_NOMEM, "host allocation failed");
    p->dim = dim;
    p->macro = macro;
    p->levels = levels;
    p->coarse = coarse_level;
    p->inc.assign(inclusions, inclusions + ninclusions);
    p->mu.assign(mu, mu + nphase);
    p->mu.resize(256, 1.0);
    p->nphase = nphase;
    if (opt) p->opt = *opt;
    else iss_default_options(&p->opt);
    if (elem_phase) {
        const int64_t ne = (dim == 3 ? n * n * n * 6 : n * n * 2);
        for (int64_t e = 0; e < ne; ++e)
            if (elem_phase[e] >= nphase) {
                delete p;
                return fail(ISS_E_INVAL, "element phase out of range");
            }
        if (p->opt.coarse_mu != ISS_COARSE_MU_AVERAGE) {
            delete p;
            return fail(ISS_E_INVAL, "per-element phases need ISS_COARSE_MU_AVERAGE (no geometry to rediscretise)");
        }
        p->elem_in.assign(elem_phase, elem_phase + ne);
    }
    {
        const char* g = std::getenv("ISS_VCYCLE_GRAPH");
        p->use_graphs = !(g && std::strcmp(g, "0") == 0);
    }
    if (p->opt.nu1 < 0 || p->opt.nu2 < 0 || p->opt.nu_inc < 0 || !(p->opt.stab_beta > 0) || p->opt.restart < 1 ||
        (p->opt.outer != ISS_OUTER_RICHARDSON && p->opt.outer != ISS_OUTER_FGMRES) ||
        (p->opt.coarse_mu != ISS_COARSE_MU_CENTROID && p->opt.coarse_mu != ISS_COARSE_MU_AVERAGE) ||
        p->opt.coarse_form < -1 || p->opt.coarse_form > 2 || p->opt.mid_form < -1 || p->opt.mid_form > 2 ||
        p->opt.merge_max_n < 0 || p->opt.spec_wide_min < 0 || p->opt.cycles < 1 || p->opt.cycles > 16 ||
        !(p->opt.f16_rms > 0) || !(p->opt.f16_rms < 65504.0) ||
        (p->opt.bc != ISS_BC_NOSLIP && p->opt.bc != ISS_BC_FREESLIP) || p->opt.split_align < 0 ||
        p->opt.split_align > 64 ||
        (p->opt.coarse_solver != ISS_COARSE_DIRECT && p->opt.coarse_solver != ISS_COARSE_MINRES) ||
        p->opt.minres_iters < 1 || p->opt.minres_iters > 1000 || p->opt.minres_cg < 0 || p->opt.minres_cg > 100) {
        delete p;
        return fail(ISS_E_INVAL, "bad options");
    }
    int rc = ISS_OK;
    do {
        {
            hipError_t e = hipGetDevice(&p->device);
            if (e != hipSuccess) { rc = fail(ISS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e)); break; }
            if ((rc = scratch_address(p->device, &p->scratch_dev))) break;
        }
        std::vector<double> imu(256);
        std::vector<float> mu32(256), imu32(256);
        for (int i = 0; i < 256; ++i) {
            imu[i] = 1.0 / p->mu[i];
            mu32[i] = (float)p->mu[i];
            imu32[i] = (float)imu[i];
        }
        if ((rc = dev_upload(p, &p->d_mu64, p->mu.data(), 256))) break;
        if ((rc = dev_upload(p, &p->d_imu64, imu.data(), 256))) break;
        if ((rc = dev_upload(p, &p->d_mu32, mu32.data(), 256))) break;
        if ((rc = dev_upload(p, &p->d_imu32, imu32.data(), 256))) break;
        if ((rc = dev_alloc(p, (void**)&p->d_partial, 1024 * 64 * sizeof(double)))) break;
        if ((rc = dev_alloc(p, (void**)&p->d_red, 64 * sizeof(double)))) break;
        if ((rc = dev_alloc(p, (void**)&p->d_flag, 256))) break;
        if ((rc = dev_alloc(p, (void**)&p->d_f16mul, 8 * sizeof(double)))) break;
        if (hipHostMalloc((void**)&p->h_pinned, 8192 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            rc = fail(ISS_E_NOMEM, "pinned host allocation failed");
            break;
        }
        if (dim == 3) {
            if ((rc = build_tables<3>(p->t3))) break;
            ElemTables<3, float> f;
            to_float<3>(p->t3, f);
            hipError_t e = upload_tables(3, &p->t3, sizeof(p->t3), &f, sizeof(f));
            if (e != hipSuccess) { rc = fail(ISS_E_HIP, std::string("upload tables: ") + hipGetErrorString(e)); break; }
        } else {
            if ((rc = build_tables<2>(p->t2))) break;
            ElemTables<2, float> f;
            to_float<2>(p->t2, f);
            hipError_t e = upload_tables(2, &p->t2, sizeof(p->t2), &f, sizeof(f));
            if (e != hipSuccess) { rc = fail(ISS_E_HIP, std::string("upload tables: ") + hipGetErrorString(e)); break; }
        }
        p->lv.resize(levels + 1);
        for (int l = levels; l >= coarse_level && rc == ISS_OK; --l) {
            if (l == levels || p->opt.coarse_mu == ISS_COARSE_MU_CENTROID) {
                if (dim == 3) centroid_phases<3>(p, l); else centroid_phases<2>(p, l);
            } else {
                if (dim == 3) averaged_viscosity<3>(p, l); else averaged_viscosity<2>(p, l);
            }
            rc = (dim == 3) ? setup_level<3>(p, l) : setup_level<2>(p, l);
        }
        if (rc) break;
        // Scales of the FP16 V-cycle: S = diag(sig_u, sig_p) makes the
        // diagonal of the finest isoviscous rows one for the viscosity
        // sqrt(mu_min mu_max) (the geometric middle of the phases).
        {
            double mlo = 1e300, mhi = 0;
            for (int i = 0; i < nphase; ++i) { mlo = std::min(mlo, mu[i]); mhi = std::max(mhi, mu[i]); }
            const double mref = std::sqrt(mlo * mhi);
            const LevelView& F = p->lv[levels].v;
            const double svis0 = dim == 3 ? p->t3.Svis[0][0][0][0] : p->t2.Svis[0][0][0][0];
            const double sc0 = dim == 3 ? p->t3.Sc[0] : p->t2.Sc[0];
            p->sig_u = 1.0 / std::sqrt(mref * F.sA * svis0);
            p->sig_p = 1.0 / std::sqrt(F.sC / mref * sc0);
            for (int l = coarse_level; l <= levels; ++l) {
                LevelView& W = p->lv[l].v16;
                W = p->lv[l].v;
                W.sA *= p->sig_u * p->sig_u;
                W.sB *= p->sig_u * p->sig_p;
                W.sC *= p->sig_p * p->sig_p;
            }
        }
        // keep element phases where the coarse matrix and the P1-P0 calls
        // (finest level) need them
        for (int l = coarse_level + 1; l < levels; ++l) std::vector<uint8_t>().swap(p->lv[l].elem_phase);
    } while (0);
    if (rc) {
        iss_problem_destroy(p);
        return rc;
    }
    *out = p;
    return ISS_OK;
}

int iss_num_vertices(const iss_problem* p, int level, int64_t* n) {
    if (!p || !n) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_level(p, level))) return rc;
    *n = p->lv[level].v.N;
    return ISS_OK;
}

int iss_vertex_class(const iss_problem* p, int level, uint8_t* cls, int64_t* ninterface,
                     int64_t* nboundary) {
    if (!p) return fail(ISS_E_INVAL, "null problem");
    int rc;
    if ((rc = check_level(p, level))) return rc;
    const Level& L = p->lv[level];
    if (cls) std::memcpy(cls, L.cls.data(), L.cls.size());
    if (ninterface) *ninterface = L.ninterface;
    if (nboundary) *nboundary = L.nboundary;
    return ISS_OK;
}

int iss_rhs_buoyancy(iss_problem* p, int level, const int* phases, int nbuoyant, double rho,
                     double* b, iss_stream_t stream) {
    if (!p || !b || (nbuoyant > 0 && !phases)) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_level(p, level))) return rc;
    if (level != p->levels && p->opt.coarse_mu != ISS_COARSE_MU_CENTROID)
        return fail(ISS_E_INVAL, "buoyancy load needs the finest level (coarse phases are viscosity bins)");
    hipStream_t s = (hipStream_t)stream;
    uint8_t flag[256] = {0};
    for (int i = 0; i < nbuoyant; ++i) {
        if (phases[i] < 0 || phases[i] > 253) return fail(ISS_E_INVAL, "bad buoyant phase");
        flag[phases[i]] = 1;
    }
    ISS_HIP(hipStreamSynchronize(s));
    ISS_HIP(hipMemcpy(p->d_flag, flag, 256, hipMemcpyHostToDevice));
    const Level& L = p->lv[level];
    ISS_HIP(k_fill(PREC_F64, b, (int64_t)(p->dim + 1) * L.v.N, 0.0, s));
    double vol = 1.0;
    for (int a = 0; a < p->dim; ++a) vol /= L.v.n;
    vol /= (p->dim == 3 ? 6.0 : 2.0);
    ISS_HIP(k_rhs_buoyancy(L.v, p->d_flag, rho, vol, b, s));
    ISS_HIP(hipStreamSynchronize(s));   // flag buffer is reused by the next call
    return ISS_OK;
}

int iss_rhs_nodal_force(iss_problem* p, int level, const double* f, double* b, iss_stream_t stream) {
    if (!p || !f || !b) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_level(p, level))) return rc;
    const Level& L = p->lv[level];
    double vol = 1.0;
    for (int a = 0; a < p->dim; ++a) vol /= L.v.n;
    vol /= (p->dim == 3 ? 6.0 : 2.0);
    ISS_HIP(k_rhs_nodal_force(L.v, f, vol, b, (hipStream_t)stream));
    return ISS_OK;
}

int iss_num_elements(const iss_problem* p, int64_t* ne) {
    if (!p || !ne) return fail(ISS_E_INVAL, "null argument");
    const Level& L = p->lv[p->levels];
    *ne = (int64_t)L.elem_phase.size();
    return ISS_OK;
}

// the device copy of the finest level's element phases, and the argument
// checks shared by the P1-P0 calls
static int p1p0_prepare(iss_problem* p, double gamma) {
    if (!(gamma > 0) || !std::isfinite(gamma)) return fail(ISS_E_INVAL, "gamma must be positive and finite");
    const Level& L = p->lv[p->levels];
    if ((int64_t)L.elem_phase.size() < L.v.N)
        return fail(ISS_E_INVAL, "P1-P0 needs at least as many elements as vertices (3D, or 2D with n >= 3)");
    if (!p->d_eph) {
        int rc = dev_upload(p, &p->d_eph, L.elem_phase.data(), L.elem_phase.size());
        if (rc) return rc;
    }
    return ISS_OK;
}

int iss_p1p0_apply(iss_problem* p, int form, double gamma, const double* x, double* y, iss_stream_t stream) {
    if (!p || !x || !y) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_form(form)) || (rc = p1p0_prepare(p, gamma))) return rc;
    ISS_HIP(k_p1p0_apply(p->lv[p->levels].v, form, p->d_eph, gamma, x, y, (hipStream_t)stream));
    return ISS_OK;
}

int iss_p1p0_flux(iss_problem* p, double gamma, const double* x, double* flux, iss_stream_t stream) {
    if (!p || !x || !flux) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = p1p0_prepare(p, gamma))) return rc;
    ISS_HIP(k_p1p0_flux(p->lv[p->levels].v, p->d_eph, gamma, x, flux, (hipStream_t)stream));
    return ISS_OK;
}

int iss_apply(iss_problem* p, int form, int block, int level, int prec, const void* x, void* y,
              iss_stream_t stream) {
    if (!p || !x || !y) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    if (block != ISS_VELOCITY_ONLY && block != ISS_FULL_STOKES) return fail(ISS_E_INVAL, "bad block");
    ISS_HIP(k_apply(p->lv[level].v, form, block, MODE_APPLY, prec, x, nullptr, y, (hipStream_t)stream));
    return ISS_OK;
}

int iss_residual(iss_problem* p, int form, int level, int prec, const void* x, const void* b, void* r,
                 double* norms, iss_stream_t stream) {
    if (!p || !x || !b || !r) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Level& L = p->lv[level];
    ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_RESID, prec, x, b, r, s));
    if (norms) {
        double sq[4];
        if ((rc = field_norms(p, prec, r, L.v.N, p->dim + 1, sq, s))) return rc;
        for (int f = 0; f <= p->dim; ++f) norms[f] = std::sqrt(sq[f]);
        norms[p->dim + 1] = total_norm(sq, p->dim + 1);
    }
    return ISS_OK;
}

int iss_smooth(iss_problem* p, int form, int level, int prec, int nsteps, void* x, const void* b,
               iss_stream_t stream) {
    if (!p || !x || !b || nsteps < 0) return fail(ISS_E_INVAL, "bad argument");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    if ((rc = ensure_work(p, level, prec))) return rc;
    Level& L = p->lv[level];
    const hipStream_t s = (hipStream_t)stream;
    const int nf = p->dim + 1;
    void *xs, *bs, *ws;
    split_buffers(p, level, prec, &xs, &bs, &ws);
    ISS_HIP(k_split(L.v, prec, nf, b, bs, SPLIT_PACK, s));
    ISS_HIP(k_split(L.v, prec, nf, x, xs, SPLIT_PACK, s));
    for (int i = 0; i < nsteps; ++i)
        ISS_HIP(k_smooth_step(L.v, form, prec, p->opt.omega, xs, bs, ws, i == 0, s));
    ISS_HIP(k_split(L.v, prec, nf, xs, x, SPLIT_UNPACK, s));
    return ISS_OK;
}

int iss_smooth_noalloc(iss_problem* p, int form, int level, int prec, int nsteps, void* x, const void* b,
                       iss_stream_t stream) {
    if (!p || !x || !b || nsteps < 0) return fail(ISS_E_INVAL, "bad argument");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    Level& L = p->lv[level];
    const int nf = p->dim + 1;
    const size_t vec = (size_t)nf * L.v.Ns * prec_bytes(prec);
    if (3 * vec > (size_t)ISS_NOALLOC_SCRATCH_BYTES)
        return fail(ISS_E_INVAL, "level too large for the no-allocation scratch (" +
                                     std::to_string(3 * vec) + " > " +
                                     std::to_string((size_t)ISS_NOALLOC_SCRATCH_BYTES) + " bytes)");
    if (!p->scratch_dev) return fail(ISS_E_HIP, "no-allocation scratch address not resolved");
    int cur = -1;
    ISS_HIP(hipGetDevice(&cur));
    if (cur != p->device) return fail(ISS_E_INVAL, "call on another device than the problem's");
    const hipStream_t s = (hipStream_t)stream;
    // the same steps as iss_smooth on the device-resident scratch; the
    // first step clears the pressure correction field with a fill kernel
    char* base = (char*)p->scratch_dev;
    void* xs = base;
    void* bs = base + vec;
    void* ws = base + 2 * vec;
    ISS_HIP(k_split(L.v, prec, nf, b, bs, SPLIT_PACK, s));
    ISS_HIP(k_split(L.v, prec, nf, x, xs, SPLIT_PACK, s));
    for (int i = 0; i < nsteps; ++i)
        ISS_HIP(k_smooth_step(L.v, form, prec, p->opt.omega, xs, bs, ws, i == 0, s));
    ISS_HIP(k_split(L.v, prec, nf, xs, x, SPLIT_UNPACK, s));
    return ISS_OK;
}

int iss_smooth_timed(iss_problem* p, int form, int level, int prec, int nsteps, void* x, const void* b,
                     iss_stream_t stream, double* ms) {
    if (!p || !x || !b || !ms || nsteps < 1) return fail(ISS_E_INVAL, "bad argument");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    if ((rc = ensure_work(p, level, prec))) return rc;
    Level& L = p->lv[level];
    const hipStream_t s = (hipStream_t)stream;
    const int nf = p->dim + 1, nph = 2 * nf;
    void *xs, *bs, *ws;
    split_buffers(p, level, prec, &xs, &bs, &ws);
    PhaseTimer tm{};
    hipEvent_t st0 = nullptr, st1 = nullptr;
    auto cleanup = [&]() {
        for (int q = 0; q < 8; ++q) {
            if (tm.begin[q]) (void)hipEventDestroy(tm.begin[q]);
            if (tm.end[q]) (void)hipEventDestroy(tm.end[q]);
        }
        if (st0) (void)hipEventDestroy(st0);
        if (st1) (void)hipEventDestroy(st1);
    };
    hipError_t e = hipSuccess;
    for (int q = 0; q < nph && e == hipSuccess; ++q) {
        e = hipEventCreate(&tm.begin[q]);
        if (e == hipSuccess) e = hipEventCreate(&tm.end[q]);
    }
    if (e == hipSuccess) e = hipEventCreate(&st0);
    if (e == hipSuccess) e = hipEventCreate(&st1);
    if (e != hipSuccess) { cleanup(); return fail(ISS_E_HIP, hipGetErrorString(e)); }
    double phase_ms = 0, step_ms = 0;
    int nphase = 0;
    e = k_split(L.v, prec, nf, b, bs, SPLIT_PACK, s);
    if (e == hipSuccess) e = k_split(L.v, prec, nf, x, xs, SPLIT_PACK, s);
    for (int i = 0; i < nsteps && e == hipSuccess; ++i) {
        e = hipEventRecord(st0, s);
        if (e == hipSuccess) e = k_smooth_step(L.v, form, prec, p->opt.omega, xs, bs, ws, i == 0, s, &tm);
        if (e == hipSuccess) e = hipEventRecord(st1, s);
        if (e == hipSuccess) e = hipEventSynchronize(st1);
        float t = 0;
        for (int q = 0; q < tm.used && e == hipSuccess; ++q) {
            e = hipEventElapsedTime(&t, tm.begin[q], tm.end[q]);
            phase_ms += t;
            ++nphase;
        }
        if (e == hipSuccess) e = hipEventElapsedTime(&t, st0, st1);
        step_ms += t;
    }
    if (e == hipSuccess) e = k_split(L.v, prec, nf, xs, x, SPLIT_UNPACK, s);
    cleanup();
    if (e != hipSuccess) return fail(ISS_E_HIP, hipGetErrorString(e));
    ms[0] = phase_ms / std::max(1, nphase);
    ms[1] = step_ms / nsteps;
    return ISS_OK;
}

int iss_restrict(iss_problem* p, int level, int prec, const void* rf, void* rc_, iss_stream_t stream) {
    if (!p || !rf || !rc_) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    if (level == p->coarse) return fail(ISS_E_INVAL, "no coarser level");
    ISS_HIP(k_restrict(p->lv[level].v, p->lv[level - 1].v, prec, rf, rc_, (hipStream_t)stream));
    return ISS_OK;
}

int iss_prolong_add(iss_problem* p, int level, int prec, const void* ec, void* xf, iss_stream_t stream) {
    if (!p || !ec || !xf) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_prec(prec)) || (rc = check_level(p, level))) return rc;
    if (level == p->coarse) return fail(ISS_E_INVAL, "no coarser level");
    ISS_HIP(k_prolong_add(p->lv[level].v, p->lv[level - 1].v, prec, ec, xf, (hipStream_t)stream));
    return ISS_OK;
}

int iss_coarse_solve(iss_problem* p, int form, const double* b, double* x, iss_stream_t stream) {
    if (!p || !b || !x) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_form(form))) return rc;
    return coarse_solve(p, form, PREC_F64, b, x, (hipStream_t)stream);
}

int iss_vcycle(iss_problem* p, int form, int prec, void* x, const void* b, iss_stream_t stream) {
    if (!p || !x || !b) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec))) return rc;
    return vcycle(p, p->levels, form, prec, x, b, false, (hipStream_t)stream);
}

int iss_solve(iss_problem* p, int form, int prec, double rtol, int maxit, double* x, const double* b,
              iss_solve_info* info, iss_stream_t stream) {
    if (!p || !x || !b) return fail(ISS_E_INVAL, "null argument");
    if (!(rtol > 0) || maxit < 0) return fail(ISS_E_INVAL, "need rtol > 0 and maxit >= 0");
    int rc;
    if ((rc = check_form(form)) || (rc = check_prec(prec))) return rc;
    return solve(p, form, prec, rtol, maxit, x, b, info, (hipStream_t)stream);
}

int iss_asymptotic_rate(iss_problem* p, int form, int iters, double* x, double* rates, iss_stream_t stream) {
    if (!p || !x || !rates || iters < 1) return fail(ISS_E_INVAL, "bad argument");
    int rc;
    if ((rc = check_form(form))) return rc;
    const int l = p->levels, D = p->dim;
    Level& L = p->lv[l];
    const int64_t N = L.v.N, n = (int64_t)(D + 1) * N;
    const hipStream_t s = (hipStream_t)stream;
    if (!p->d_rate) {
        if ((rc = work_alloc(p, (void**)&p->d_rate, (size_t)2 * n * sizeof(double)))) return rc;
        ISS_HIP(k_fill(PREC_F64, p->d_rate, n, 0.0, s));
    }
    const double* zero = p->d_rate;
    double* y = p->d_rate + n;
    double sq[4];
    ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_APPLY, PREC_F64, x, nullptr, y, s));
    if ((rc = field_norms(p, PREC_F64, y, N, D + 1, sq, s))) return rc;
    double r0 = total_norm(sq, D + 1);
    if (!(r0 > 0) || !std::isfinite(r0)) return fail(ISS_E_INVAL, "K x of the initial iterate is zero or not finite");
    ISS_HIP(k_scale(x, 1.0 / r0, x, n, s));
    for (int it = 0; it < iters; ++it) {
        // one stationary cycle on K x = 0, then the constant pressure (the
        // kernel of K, untouched by the cycle) is removed so that the
        // rescaling cannot let it grow
        if ((rc = vcycle(p, l, form, PREC_F64, x, zero, false, s))) return rc;
        ISS_HIP(k_field_sum(x + (int64_t)D * N, N, p->d_partial, p->d_red, s));
        ISS_HIP(k_sub_mean(x + (int64_t)D * N, N, p->d_red, s));
        ISS_HIP(k_apply(L.v, form, BLOCK_FULL, MODE_APPLY, PREC_F64, x, nullptr, y, s));
        if ((rc = field_norms(p, PREC_F64, y, N, D + 1, sq, s))) return rc;
        const double r1 = total_norm(sq, D + 1);
        rates[it] = r1;            // ||K x|| was 1 before the cycle
        if (!(r1 > 0) || !std::isfinite(r1)) return fail(ISS_E_DIVERGED, "rate iteration lost its iterate");
        ISS_HIP(k_scale(x, 1.0 / r1, x, n, s));
    }
    ISS_HIP(hipStreamSynchronize(s));
    return ISS_OK;
}

int iss_dot(iss_problem* p, const double* a, const double* b, int64_t n, double* out, iss_stream_t stream) {
    if (!p || !a || !b || !out || n < 0) return fail(ISS_E_INVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    ISS_HIP(k_multidot(a, 0, 1, b, n, p->d_partial, p->d_red, s));
    ISS_HIP(hipMemcpyAsync(p->h_pinned, p->d_red, sizeof(double), hipMemcpyDeviceToHost, s));
    ISS_HIP(hipStreamSynchronize(s));
    *out = p->h_pinned[0];
    return ISS_OK;
}

int iss_workspace_bytes(const iss_problem* p, int prec, size_t* bytes) {
    if (!p || !bytes) return fail(ISS_E_INVAL, "null argument");
    int rc;
    if ((rc = check_prec(prec))) return rc;
    const int nf = p->dim + 1;
    size_t t = 0;
    for (int l = p->coarse; l <= p->levels; ++l) {       // work vectors of every level
        const LevelView& V = p->lv[l].v;
        t += 3 * ws_round((size_t)nf * V.N * prec_bytes(prec));
        t += ws_round((size_t)3 * nf * V.Ns * prec_bytes(prec));
    }
    const size_t n = (size_t)nf * p->lv[p->levels].v.N;
    const size_t m = (size_t)std::max(1, p->opt.restart);
    t += ws_round((m + 1) * n * 8) + ws_round(m * n * 8) + 2 * ws_round(n * 8) + ws_round((2 * m + 4) * 8);
    t += ws_round(2 * n * 8);                              // rate measurement
    *bytes = t;
    return ISS_OK;
}

int iss_bind_workspace(iss_problem* p, void* dev_ptr, size_t bytes) {
    if (!p || !dev_ptr) return fail(ISS_E_INVAL, "null argument");
    if (((uintptr_t)dev_ptr & (WS_ALIGN - 1)) != 0) return fail(ISS_E_INVAL, "workspace must be 256-byte aligned");
    bool used = p->d_V || p->d_rate || p->ws_base;
    for (const auto& L : p->lv)
        for (int q = 0; q < NPREC; ++q) used = used || L.w_x[q] || L.w_s[q];
    if (used) return fail(ISS_E_INVAL, "bind the workspace before the first call that needs work buffers");
    p->ws_base = (char*)dev_ptr;
    p->ws_size = bytes;
    p->ws_used = 0;
    return ISS_OK;
}

int iss_launch_counts(iss_problem* p, int64_t* counts, int n, int reset) {
    if (!p || !counts || n < ISS_L_KINDS) return fail(ISS_E_INVAL, "need a problem and ISS_L_KINDS counters");
    for (int k = 0; k < ISS_L_KINDS; ++k) counts[k] = p->launch_count[k];
    if (reset)
        for (int k = 0; k < ISS_L_KINDS; ++k) p->launch_count[k] = 0;
    return ISS_OK;
}

// ---- learned band correction ------------------------------------------------

int iss_net_create(iss_problem* p, iss_net** out) {
    if (!p || !out) return fail(ISS_E_INVAL, "null argument");
    *out = nullptr;
    if (p->dim != 3) return fail(ISS_E_INVAL, "the band correction network is 3D only");
    if (p->opt.bc != ISS_BC_NOSLIP) return fail(ISS_E_INVAL, "the band correction network is trained for no-slip");
    const Level& L = p->lv[p->levels];
    const int n = L.v.n;
    const int64_t n1 = n + 1, N = L.v.N;
    // band: Chebyshev distance <= 2 from an interface vertex
    std::vector<uint8_t> band(N, 0);
    for (int64_t v = 0; v < N; ++v) {
        if (!(L.cls[v] & 1)) continue;
        const int i = (int)(v % n1), j = (int)((v / n1) % n1), k = (int)(v / (n1 * n1));
        for (int dk = -2; dk <= 2; ++dk)
            for (int dj = -2; dj <= 2; ++dj)
                for (int di = -2; di <= 2; ++di) {
                    const int a = i + di, b = j + dj, c = k + dk;
                    if (a < 0 || b < 0 || c < 0 || a > n || b > n || c > n) continue;
                    band[a + n1 * (b + n1 * c)] = 1;
                }
    }
    // max incident viscosity per vertex
    std::vector<double> mumax(N, 0.0);
    for (int64_t v = 0; v < N; ++v)
        if (L.h_vphase[v] != SPECIAL) mumax[v] = L.mu_tab[L.h_vphase[v]];
    constexpr int NS = KuhnTables<3>::NS;
    for (size_t q = 0; q < L.h_spec.size(); ++q) {
        double mx = 0;
        for (int sl = 0; sl < NS; ++sl) {
            const int ph = L.h_eph[q * NS + sl];
            if (ph != OUTSIDE) mx = std::max(mx, L.mu_tab[ph]);
        }
        mumax[L.h_spec[q]] = mx;
    }
    NetSetup su;
    su.n = n;
    su.N = N;
    su.nvec = 4 * N;
    su.beta = p->opt.stab_beta;
    for (int64_t v = 0; v < N; ++v)
        if (band[v]) {
            su.band.push_back((int32_t)v);
            su.static_feat.push_back((float)(std::log10(mumax[v] > 0 ? mumax[v] : 1.0) / 4.0));
            su.static_feat.push_back((L.cls[v] & 1) ? 1.0f : 0.0f);
        }
    iss_net* net = new (std::nothrow) iss_net();
    if (!net) return fail(ISS_E_NOMEM, "host allocation failed");
    net->p = p;
    hipError_t e = net_create(su, &net->impl);
    if (e != hipSuccess) {
        delete net;
        return fail(ISS_E_HIP, std::string("net create: ") + hipGetErrorString(e));
    }
    p->nets.push_back(net);
    *out = net;
    return ISS_OK;
}

void iss_net_destroy(iss_net* net) {
    if (!net) return;
    if (net->p) {
        if (net->p->net == net) net->p->net = nullptr;
        auto& v = net->p->nets;
        v.erase(std::remove(v.begin(), v.end(), net), v.end());
    }
    net_destroy(net->impl);
    delete net;
}

int iss_net_save_input(iss_net* net, uint16_t* dst, iss_stream_t stream) {
    if (!net || !dst) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_save_input(net->impl, dst, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_load_input(iss_net* net, const uint16_t* src, iss_stream_t stream) {
    if (!net || !src) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_load_input(net->impl, src, (hipStream_t)stream));
    return ISS_OK;
}

int iss_axpby(double a, const double* x, double b, double* y, int64_t n, iss_stream_t stream) {
    if (!x || !y || n < 0) return fail(ISS_E_INVAL, "bad argument");
    if (n == 0) return ISS_OK;
    ISS_HIP(k_axpby(y, a, x, b, n, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_info(const iss_net* net, int64_t* band_size, int64_t* num_params) {
    if (!net) return fail(ISS_E_INVAL, "null net");
    if (band_size) *band_size = net_band_size(net->impl);
    if (num_params) *num_params = net_num_params(net->impl);
    return ISS_OK;
}

int iss_net_band(const iss_net* net, int32_t* band) {
    if (!net || !band) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_copy_band(net->impl, band));
    return ISS_OK;
}

int iss_net_set_weights(iss_net* net, const float* w, iss_stream_t stream) {
    if (!net || !w) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_set_weights(net->impl, w, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_features(iss_net* net, const double* r, double* scales, iss_stream_t stream) {
    if (!net || !r) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_features(net->impl, r, scales, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_forward(iss_net* net, float* y, iss_stream_t stream) {
    if (!net) return fail(ISS_E_INVAL, "null net");
    ISS_HIP(net_forward(net->impl, y, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_targets(iss_net* net, const double* err, float* t, iss_stream_t stream) {
    if (!net || !err || !t) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_targets(net->impl, err, t, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_backward(iss_net* net, const float* t, float* grad, double* loss, iss_stream_t stream) {
    if (!net || !grad) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_backward(net->impl, t, grad, loss, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_correction(iss_net* net, double* c, iss_stream_t stream) {
    if (!net || !c) return fail(ISS_E_INVAL, "null argument");
    if (!net->p) return fail(ISS_E_INVAL, "the problem of this network has been destroyed");
    const Level& L = net->p->lv[net->p->levels];
    ISS_HIP(net_output_correction(net->impl, c, (int64_t)(net->p->dim + 1) * L.v.N, (hipStream_t)stream));
    return ISS_OK;
}

int iss_net_output_grad(iss_net* net, const double* dldc, double factor, iss_stream_t stream) {
    if (!net || !dldc) return fail(ISS_E_INVAL, "null argument");
    ISS_HIP(net_output_grad(net->impl, dldc, factor, (hipStream_t)stream));
    return ISS_OK;
}

int iss_adam_step(int64_t n, float* w, float* m, float* v, const float* g, float lr, int step,
                  iss_stream_t stream) {
    if (!w || !m || !v || !g || n < 0 || step < 1) return fail(ISS_E_INVAL, "bad argument");
    ISS_HIP(net_adam(n, w, m, v, g, lr, step, (hipStream_t)stream));
    return ISS_OK;
}

int iss_problem_set_net(iss_problem* p, iss_net* net) {
    if (net && !net->p) return fail(ISS_E_INVAL, "the problem of this network has been destroyed");
    if (!p) return fail(ISS_E_INVAL, "null problem");
    if (net && net->p != p) return fail(ISS_E_INVAL, "net belongs to another problem");
    p->net = net;
    return ISS_OK;
}

}  // extern "C"
