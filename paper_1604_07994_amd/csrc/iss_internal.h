// Internal declarations shared by the host setup/solver code and the HIP
// kernels of the Stokes hot path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "iss_geometry.h"

namespace iss {

constexpr uint8_t SPECIAL = 255;   // vertex phase byte: needs the element loop
constexpr uint8_t OUTSIDE = 255;   // incident-element phase: outside the domain

enum { FORM_GRADIENT = 0, FORM_STRAIN = 1, FORM_INTERFACE = 2 };
enum { BLOCK_VEL = 0, BLOCK_FULL = 1 };
enum { MODE_APPLY = 0, MODE_RESID = 1 };
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_F16 = 3, NPREC = 4 };   // storage; BF16, FP16 computed in FP32
inline int prec_bytes(int prec) { return prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 2); }

// Per-level data as seen by the kernels (all pointers are device pointers).
struct LevelView {
    int dim;
    int n;                   // cells per axis; vertices 0..n per axis
    int64_t N;               // (n+1)^dim
    int64_t sy, sz;          // strides of j and k (sz = 0 in 2D)
    const uint8_t* vphase;   // per vertex: phase, or SPECIAL
    const int32_t* spec;     // special vertices grouped by colour
    const uint8_t* spec_eph; // per special vertex: phase of each slot
    int64_t spec_off[5];     // colour c occupies [spec_off[c], spec_off[c+1])
    int64_t spec_mid[4];     // colour c: boundary rows before spec_mid[c], interior ones after
    const double* mu64;      // viscosity per phase
    const double* imu64;     // 1 / viscosity per phase
    const float* mu32;
    const float* imu32;
    double sA, sB, sC;       // h^(d-2), h^(d-1), beta h^d
    // colour-split layout used inside smoothing calls: vertex (i, j, k) at
    // k Pp + j Rp + (i mod (d+1)) q + i div (d+1); Ns entries per field
    int q, Rp;
    int64_t Pp, Ns;
    const uint8_t* vphase_s; // phase bytes in the split layout (padding SPECIAL)
    // smoother launch shapes (host side): merged colour phases up to this n,
    // 256-thread pressure special groups above this list length
    int merge_max_n;
    int64_t spec_wide_min;
    int64_t* launch_count;   // host counters per iss_launch_kind, or null
    int freeslip;            // 0: no-slip (every boundary velocity fixed);
                             // 1: free-slip (the normal component fixed)
};

enum { SPLIT_PACK = 0, SPLIT_UNPACK = 1 };

// Kernel launchers (iss_kernels.hip).  `prec` selects double / float
// vectors.  Each returns hipSuccess or the launch error.
hipError_t upload_tables(int dim, const void* t64, size_t bytes64, const void* t32,
                         size_t bytes32);
hipError_t k_apply(const LevelView& L, int form, int block, int mode, int prec,
                   const void* x, const void* b, void* y, hipStream_t s);
// events around the bulk velocity colour-phase launches of a step (at most
// 2 (d+1)); `used` counts the pairs recorded by the last step
struct PhaseTimer {
    hipEvent_t begin[8], end[8];
    int used = 0;
};
// one Uzawa step on split-layout vectors xs, bs (d+1 fields of Ns each);
// ws holds d+1 split fields of scratch.  first_step: the first step of a
// sequence on these buffers (clears the pressure correction field of ws;
// later steps rely on the previous step having left it cleared).  tm
// (optional) times the bulk velocity colour phases
hipError_t k_smooth_step(const LevelView& L, int form, int prec, double omega, void* xs,
                         const void* bs, void* ws, bool first_step, hipStream_t s, PhaseTimer* tm = nullptr);
// canonical <-> split copy of nf fields (dir SPLIT_PACK: canonical in, split
// out with zero padding; SPLIT_UNPACK: split in, canonical out)
hipError_t k_split(const LevelView& L, int prec, int nf, const void* in, void* out, int dir,
                   hipStream_t s);
hipError_t k_restrict(const LevelView& Lf, const LevelView& Lc, int prec, const void* rf,
                      void* rc, hipStream_t s);
hipError_t k_prolong_add(const LevelView& Lf, const LevelView& Lc, int prec, const void* ec,
                         void* xf, hipStream_t s);
hipError_t k_fill(int prec, void* x, int64_t n, double value, hipStream_t s);
hipError_t k_convert(int prec_in, const void* in, int prec_out, void* out, int64_t n,
                     hipStream_t s);
// sums of squares per field (nf fields of length N) -> out[0..nf-1] (device,
// FP64), using `partial` (device, >= 1024 * nf doubles) as scratch.
hipError_t k_field_sumsq(int prec, const void* x, int64_t N, int nf, double* partial,
                         double* out, hipStream_t s);
// out[0] = sum of the n entries of x (partial: >= 1024 doubles); x -= sum / n
hipError_t k_field_sum(const double* x, int64_t n, double* partial, double* out, hipStream_t s);
hipError_t k_sub_mean(double* x, int64_t n, const double* sum, hipStream_t s);
// out[i] = sum_e V_i[e] w[e] for i < k (V_i = V + i * ldv), and out[k] = w.w
// if with_self; partial holds 65536 doubles.
hipError_t k_multidot(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                      double* partial, double* out, hipStream_t s, int with_self = 0);
// Delayed classical Gram-Schmidt: out[0..k) = V^T a, out[k..2k) = V^T b,
// out[2k] = a.a, out[2k+1] = a.b, out[2k+2] = b.b (partial: 65536 doubles)
hipError_t k_dots2(const double* V, int64_t ldv, int k, const double* a, const double* b, int64_t n,
                   double* partial, double* out, hipStream_t s);
// V_k = (V_k - sum_i c_i V_i) inv_alpha;  V_{k+1} = (w - sum_i d_i V_i - e V_k) inv_s
hipError_t k_dcgs_update(double* V, int64_t ldv, int k, const double* c, const double* d, const double* w,
                         double inv_alpha, double ecoef, double inv_s, int64_t n, hipStream_t s);
// y += alpha * sum_i c[i] X_i  (c on device)
hipError_t k_multiaxpy(double* y, const double* X, int64_t ldx, int k, const double* c,
                       double alpha, int64_t n, hipStream_t s);
// y = a * x
hipError_t k_scale(double* y, double a, const double* x, int64_t n, hipStream_t s);
hipError_t k_axpby(double* y, double a, const double* x, double b, int64_t n,
                   hipStream_t s);
// per-field multipliers of gathered / scattered entries (entry e of a
// vector with fields of N entries belongs to field e / N); on = 0: none
struct FieldMul {
    double m[4];
    int64_t N;
    int on;
};
hipError_t k_gather(int prec, const void* x, const int32_t* idx, int64_t m, double* out,
                    hipStream_t s, FieldMul fm = FieldMul{});
hipError_t k_scatter(int prec, const double* in, const int32_t* idx, int64_t m, void* x,
                     hipStream_t s, FieldMul fm = FieldMul{});
// out = in * mul[field] for nf fields of N entries between FP64 and the
// storage precision `prec` (dir 0: FP64 in, prec out; dir 1: prec in, FP64
// out); mul on the device
hipError_t k_scale_convert(int prec, int dir, const void* in, void* out, int64_t N, int nf,
                           const double* mul, hipStream_t s);
// multipliers of the scaled FP16 V-cycle from the field sums of squares of
// its FP64 input (device): gamma = target / RMS of (S v); in_mul[f] =
// gamma sig_f, out_mul[f] = sig_f / gamma (mul = [in_mul | out_mul])
hipError_t k_f16_multipliers(const double* sumsq, int nf, int64_t n, double sig_u, double sig_p, double target,
                             double* mul, hipStream_t s);
hipError_t k_dense_matvec(const double* A, int64_t m, const double* x, double* y,
                          hipStream_t s);
hipError_t k_rhs_buoyancy(const LevelView& L, const uint8_t* buoyant_flag, double rho,
                          double vol_unit, double* b, hipStream_t s);
// b = (M f_1 | .. | M f_d | 0), fixed velocity entries zero; vol = |T|
hipError_t k_rhs_nodal_force(const LevelView& L, const double* f, double vol, double* b, hipStream_t s);

// ---- Krylov coarse solver (iss_krylov.hip)
// device buffers of the coarse MINRES: (d+1) N doubles each on the coarsest
// level, st 16 doubles of scalar state, inv_d the inverse Jacobi diagonal of
// the velocity block (0 on fixed dofs) followed by 1 / w on the pressure
struct KrylovBufs {
    double* st;
    const double* inv_d;
    double* v[3];
    double* z[2];
    double* w[3];
    double* q;
    double* t;
    double* u;
    double* r;
    double* zc;
    double* pc;
    double* qc;
};
// x = MINRES_{minres_iters}(K, P; b) from x = 0 on level L (form), P^-1 =
// diag(CG_{cg_iters}(A, D_A), M_p^-1); with mod, b_u += B^T M_p^-1 b_p
// first; b (overwritten: modified, projected) and x are FP64 vectors of L
hipError_t minres_coarse(const LevelView& L, int form, const KrylovBufs& kb, int minres_iters, int cg_iters,
                         bool mod, double* b, double* x, hipStream_t s);

// ---- stabilised P1-P0 (iss_p1p0.hip), finest level L; vectors hold the
// d velocity fields of N vertices followed by one pressure per element
// (cell * d! + type); eph: the element phases (device)
hipError_t k_p1p0_apply(const LevelView& L, int form, const uint8_t* eph, double gamma, const double* x, double* y,
                        hipStream_t s);
hipError_t k_p1p0_flux(const LevelView& L, const uint8_t* eph, double gamma, const double* x, double* flux,
                       hipStream_t s);

// ---- learned band correction (iss_net.hip)
struct NetImpl;
struct NetSetup {
    int n;                               // finest level cells per axis (3D)
    int64_t N, nvec;                     // vertices, (d+1) N
    double beta;                         // stabilisation constant
    std::vector<int32_t> band;           // band vertex ids, ascending
    std::vector<float> static_feat;      // per band vertex: log10(max mu)/4, interface flag
};
hipError_t net_create(const NetSetup& s, NetImpl** out);
void net_destroy(NetImpl* n);
int64_t net_band_size(const NetImpl* n);
int64_t net_num_params(const NetImpl* n);
hipError_t net_copy_band(const NetImpl* n, int32_t* host);
hipError_t net_set_weights(NetImpl* n, const float* w, hipStream_t s);
hipError_t net_features(NetImpl* n, const double* r, double* scales_host, hipStream_t s);
hipError_t net_forward(NetImpl* n, float* y_out, hipStream_t s);
hipError_t net_targets(NetImpl* n, const double* err, float* t, hipStream_t s);
hipError_t net_backward(NetImpl* n, const float* t, float* grad, double* loss_host, hipStream_t s);
hipError_t net_adam(int64_t count, float* w, float* m, float* v, const float* g, float lr, int step,
                    hipStream_t s);
hipError_t net_correction(NetImpl* n, const double* r, double* c, int64_t nvec, hipStream_t s);
hipError_t net_output_correction(NetImpl* n, double* c, int64_t nvec, hipStream_t s);
hipError_t net_output_grad(NetImpl* n, const double* dldc, double factor, hipStream_t s);
double* net_work(NetImpl* n, int which);
// band rows of the network input (M x 8 BF16 bits) to / from caller memory
hipError_t net_save_input(NetImpl* n, uint16_t* dst, hipStream_t s);
hipError_t net_load_input(NetImpl* n, const uint16_t* src, hipStream_t s);

}  // namespace iss
