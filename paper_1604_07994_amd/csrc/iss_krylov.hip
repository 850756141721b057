// Krylov coarse-grid solver (Sec. 5): MINRES on the coarse saddle-point
// system, preconditioned block-diagonally by a Jacobi-preconditioned CG on
// the velocity block and the lumped (1/mu-weighted) pressure mass.
//
// The coarse level is small (9^3 or 17^3 lattice vertices), so the vector
// work of one MINRES or CG step -- its dot products, the scalar recurrence
// and the vector updates -- is one single-workgroup kernel: the reductions
// finish inside the workgroup and the scalars stay in device memory.  With
// fixed iteration counts a coarse solve is a fixed launch sequence (4 + 3m
// launches per MINRES step with m CG steps, the operator applies included)
// with no host synchronisation, so it is recorded into the V-cycle's HIP
// graph like the rest of the coarse part.
//
// MINRES: Paige and Saunders (SIAM J. Numer. Anal. 12, 1975), preconditioned
// form as in Elman, Silvester and Wathen (Finite Elements and Fast Iterative
// Solvers, 2005, Alg. 4.1).  CG: Hestenes and Stiefel (1952), diagonal
// preconditioner.
#include <hip/hip_runtime.h>

#include <utility>

#include "iss_internal.h"

namespace iss {

namespace {

constexpr int KWG = 1024;   // threads of the single-workgroup kernels

// scalar state of the iteration (device memory)
enum { S_GOLD = 0, S_G, S_ETA, S_COLD, S_C, S_SOLD, S_S, S_DELTA, S_RZ, S_LIVE, S_SUM, S_NST = 16 };

__device__ __forceinline__ double wg_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    __syncthreads();   // sh may still be read by a previous reduction
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < KWG / 64; ++i) s += sh[i];
    if (threadIdx.x == 0) sh[KWG / 64] = s;
    __syncthreads();
    return sh[KWG / 64];
}

// b_p -= mean(b_p) over the pressure field [dN, n)
__global__ __launch_bounds__(KWG) void k_kr_project(double* __restrict__ b, int64_t dN, int64_t n) {
    __shared__ double sh[KWG / 64 + 1];
    double acc = 0;
    for (int64_t i = dN + threadIdx.x; i < n; i += KWG) acc += b[i];
    const double mean = wg_sum(acc, sh) / (double)(n - dN);
    for (int64_t i = dN + threadIdx.x; i < n; i += KWG) b[i] -= mean;
}

// x_p -= (w . x_p) / sum(w), w the pressure weights (1 / inv_d on [dN, n))
__global__ __launch_bounds__(KWG) void k_kr_weighted_mean(double* __restrict__ x, const double* __restrict__ inv_d,
                                                          int64_t dN, int64_t n) {
    __shared__ double sh[KWG / 64 + 1];
    double a = 0, b = 0;
    for (int64_t i = dN + threadIdx.x; i < n; i += KWG) {
        const double w = 1.0 / inv_d[i];
        a += w * x[i];
        b += w;
    }
    const double wx = wg_sum(a, sh);
    const double ws = wg_sum(b, sh);
    const double m = wx / ws;
    for (int64_t i = dN + threadIdx.x; i < n; i += KWG) x[i] -= m;
}

// y_u += t_u (velocity part), the modified right-hand side r_1 + B^T M^-1 r_2
__global__ __launch_bounds__(256) void k_kr_add_vel(double* __restrict__ y, const double* __restrict__ t, int64_t dN) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < dN) y[i] += t[i];
}

// t = (0, b_p inv_w): the vector whose B^T part is B^T M^-1 b_p
__global__ __launch_bounds__(256) void k_kr_mod_vec(double* __restrict__ t, const double* __restrict__ b,
                                                    const double* __restrict__ inv_d, int64_t dN, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) t[i] = i < dN ? 0.0 : b[i] * inv_d[i];
}

// Lanczos step (or, with init, the start from v_new = b): v_new = q -
// (delta / gamma) v - (gamma / gamma_old) v_old with delta = q . z; then the
// start of the preconditioner: r = v_new_u, zc = D^-1 r, pc = zc, u = 0,
// rz = r . zc, and the pressure part of z_new = v_new_p / w.
__global__ __launch_bounds__(KWG) void k_kr_lanczos(double* __restrict__ st, int init, const double* __restrict__ q,
                                                    const double* __restrict__ z, const double* __restrict__ v,
                                                    const double* __restrict__ v_old, double* __restrict__ v_new,
                                                    double* __restrict__ z_new, const double* __restrict__ inv_d,
                                                    double* __restrict__ u, double* __restrict__ r,
                                                    double* __restrict__ zc, double* __restrict__ pc, int64_t dN,
                                                    int64_t n) {
    __shared__ double sh[KWG / 64 + 1];
    double a = 0, b = 0;
    if (!init) {
        const bool live = st[S_LIVE] != 0.0;
        double d = 0;
        for (int64_t i = threadIdx.x; i < n; i += KWG) d += q[i] * z[i];
        const double delta = wg_sum(d, sh);
        const double g = st[S_G], go = st[S_GOLD];
        a = live ? delta / g : 0.0;
        b = live ? g / go : 0.0;
        if (threadIdx.x == 0) st[S_DELTA] = delta;
    }
    double rz = 0;
    for (int64_t i = threadIdx.x; i < n; i += KWG) {
        const double vn = init ? v_new[i] : q[i] - a * v[i] - b * v_old[i];
        if (!init) v_new[i] = vn;
        if (i < dN) {
            const double zi = inv_d[i] * vn;
            r[i] = vn;
            zc[i] = zi;
            pc[i] = zi;
            u[i] = 0.0;
            rz += vn * zi;
        } else {
            z_new[i] = inv_d[i] * vn;
            r[i] = 0.0;
            zc[i] = 0.0;
            pc[i] = 0.0;
            u[i] = 0.0;
        }
    }
    rz = wg_sum(rz, sh);
    if (threadIdx.x == 0) st[S_RZ] = rz;
}

// one Jacobi-PCG step on the velocity block, qc = A pc given
__global__ __launch_bounds__(KWG) void k_kr_cg(double* __restrict__ st, const double* __restrict__ qc,
                                               const double* __restrict__ inv_d, double* __restrict__ u,
                                               double* __restrict__ r, double* __restrict__ zc,
                                               double* __restrict__ pc, int64_t dN) {
    __shared__ double sh[KWG / 64 + 1];
    double d = 0;
    for (int64_t i = threadIdx.x; i < dN; i += KWG) d += pc[i] * qc[i];
    const double pq = wg_sum(d, sh);
    const double rz = st[S_RZ];
    const double alpha = (rz != 0.0 && pq != 0.0) ? rz / pq : 0.0;
    double e = 0;
    for (int64_t i = threadIdx.x; i < dN; i += KWG) {
        u[i] += alpha * pc[i];
        const double ri = r[i] - alpha * qc[i];
        const double zi = inv_d[i] * ri;
        r[i] = ri;
        zc[i] = zi;
        e += ri * zi;
    }
    const double rz_new = wg_sum(e, sh);
    const double beta = rz != 0.0 ? rz_new / rz : 0.0;
    for (int64_t i = threadIdx.x; i < dN; i += KWG) pc[i] = zc[i] + beta * pc[i];
    if (threadIdx.x == 0) st[S_RZ] = rz_new;
}

// End of a MINRES step (or of the start, with init): z_new_u = the CG
// result, gamma_new = sqrt(z_new . v_new); the Givens recurrence, w_new =
// (z - a3 w_old - a2 w) / a1, x += c_new eta w_new, eta = -s_new eta; then
// z_new /= gamma_new for the next step.
__global__ __launch_bounds__(KWG) void k_kr_update(double* __restrict__ st, int init, int use_u,
                                                   const double* __restrict__ u, const double* __restrict__ zc,
                                                   double* __restrict__ z_new, const double* __restrict__ v_new,
                                                   const double* __restrict__ z, const double* __restrict__ w_old,
                                                   const double* __restrict__ w, double* __restrict__ w_new,
                                                   double* __restrict__ x, int64_t dN, int64_t n) {
    __shared__ double sh[KWG / 64 + 1];
    double d = 0;
    for (int64_t i = threadIdx.x; i < n; i += KWG) {
        if (i < dN) z_new[i] = use_u ? u[i] : zc[i];
        d += z_new[i] * v_new[i];
    }
    const double gn = sqrt(fmax(wg_sum(d, sh), 0.0));
    if (init) {
        for (int64_t i = threadIdx.x; i < n; i += KWG) {
            x[i] = 0.0;
            w_new[i] = 0.0;      // w and w_old of the first step
            if (gn > 0.0) z_new[i] /= gn;
        }
        if (threadIdx.x == 0) {
            st[S_G] = gn;
            st[S_GOLD] = 1.0;
            st[S_ETA] = gn;
            st[S_COLD] = st[S_C] = 1.0;
            st[S_SOLD] = st[S_S] = 0.0;
            st[S_LIVE] = gn > 0.0 ? 1.0 : 0.0;
        }
        return;
    }
    const bool live = st[S_LIVE] != 0.0;
    const double g = st[S_G], delta = st[S_DELTA], c = st[S_C], co = st[S_COLD], s = st[S_S], so = st[S_SOLD];
    const double eta = st[S_ETA];
    const double a0 = c * delta - co * s * g;
    const double a1 = sqrt(a0 * a0 + gn * gn);
    const double a2 = s * delta + co * c * g;
    const double a3 = so * g;
    const double cn = live ? a0 / a1 : c, sn = live ? gn / a1 : s;
    for (int64_t i = threadIdx.x; i < n; i += KWG) {
        if (live) {
            const double wn = (z[i] - a3 * w_old[i] - a2 * w[i]) / a1;
            w_new[i] = wn;
            x[i] += cn * eta * wn;
        }
        if (gn > 0.0) z_new[i] /= gn;
    }
    __syncthreads();
    if (threadIdx.x == 0 && live) {
        st[S_ETA] = -sn * eta;
        st[S_GOLD] = g;
        st[S_G] = gn;
        st[S_COLD] = c;
        st[S_C] = cn;
        st[S_SOLD] = s;
        st[S_S] = sn;
        st[S_LIVE] = gn > 0.0 ? 1.0 : 0.0;
    }
}

}  // namespace

hipError_t minres_coarse(const LevelView& L, int form, const KrylovBufs& kb, int minres_iters, int cg_iters,
                         bool mod, double* b, double* x, hipStream_t s) {
    const int64_t N = L.N, dN = (int64_t)L.dim * N, n = dN + N;
    const dim3 g1(1), tb(KWG);
    hipError_t e;
    if (mod) {
        // r_1 + B^T M^-1 r_2: the velocity part of K (0, M^-1 r_2)
        hipLaunchKernelGGL(k_kr_mod_vec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, kb.t, b, kb.inv_d, dN, n);
        if ((e = k_apply(L, form, BLOCK_FULL, MODE_APPLY, PREC_F64, kb.t, nullptr, kb.q, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_kr_add_vel, dim3((unsigned)((dN + 255) / 256)), dim3(256), 0, s, b, kb.q, dN);
    }
    hipLaunchKernelGGL(k_kr_project, g1, tb, 0, s, b, dN, n);
    double* v_old = kb.v[0];
    double* v = b;                   // v_1 = b
    double* v_new = kb.v[1];
    double* v_spare = kb.v[2];
    double* z = kb.z[0];
    double* z_new = kb.z[1];
    double* w_old = kb.w[0];
    double* w = kb.w[1];
    double* w_new = kb.w[2];
    auto precondition = [&](int init, const double* vn) -> hipError_t {
        hipLaunchKernelGGL(k_kr_lanczos, g1, tb, 0, s, kb.st, init, kb.q, z, v, v_old, const_cast<double*>(vn),
                           z_new, kb.inv_d, kb.u, kb.r, kb.zc, kb.pc, dN, n);
        for (int k = 0; k < cg_iters; ++k) {
            hipError_t e2 = k_apply(L, form, BLOCK_VEL, MODE_APPLY, PREC_F64, kb.pc, nullptr, kb.qc, s);
            if (e2 != hipSuccess) return e2;
            hipLaunchKernelGGL(k_kr_cg, g1, tb, 0, s, kb.st, kb.qc, kb.inv_d, kb.u, kb.r, kb.zc, kb.pc, dN);
        }
        return hipGetLastError();
    };
    // start: z_1 = P^-1 b, gamma_1, x = 0, w = w_old = 0
    if ((e = k_fill(PREC_F64, v_old, n, 0.0, s)) != hipSuccess) return e;
    if ((e = precondition(1, v)) != hipSuccess) return e;
    {
        // z_new holds z_1 after the update; w_old is cleared by init (w_new
        // argument) and w below
        hipLaunchKernelGGL(k_kr_update, g1, tb, 0, s, kb.st, 1, cg_iters > 0 ? 1 : 0, kb.u, kb.zc, z_new, v, z,
                           w_old, w, w_old, x, dN, n);
        if ((e = k_fill(PREC_F64, w, n, 0.0, s)) != hipSuccess) return e;
        std::swap(z, z_new);
    }
    for (int it = 0; it < minres_iters; ++it) {
        if ((e = k_apply(L, form, BLOCK_FULL, MODE_APPLY, PREC_F64, z, nullptr, kb.q, s)) != hipSuccess) return e;
        if ((e = precondition(0, v_new)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_kr_update, g1, tb, 0, s, kb.st, 0, cg_iters > 0 ? 1 : 0, kb.u, kb.zc, z_new, v_new, z,
                           w_old, w, w_new, x, dN, n);
        // rotate: v_old <- v, v <- v_new; z <- z_new; w_old <- w <- w_new
        double* vo = v_old;
        v_old = v;
        v = v_new;
        v_new = (vo == b) ? v_spare : vo;
        if (vo == b) v_spare = nullptr;
        std::swap(z, z_new);
        double* wo = w_old;
        w_old = w;
        w = w_new;
        w_new = wo;
    }
    hipLaunchKernelGGL(k_kr_weighted_mean, g1, tb, 0, s, x, kb.inv_d, dN, n);
    return hipGetLastError();
}

}  // namespace iss
