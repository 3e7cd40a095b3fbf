// gfx950 kernels of the MinRes slab inverse (Section 3.3, Theorems 3.8 and
// 3.10): with the temporal eigen form, A^{-1} = (V (x) I)(Z (x) M_x + I (x)
// K_x)^{-1}(W (x) I); a real eigenvalue gives the spatial system K_x +
// lambda M_x (solved exactly by the fast diagonalisation), a conjugate pair
// alpha +- i beta the 2x2 block system that Theorem 3.10 turns into the
// symmetric indefinite A_bar [x; -y] = [|b2| f; |b1| g], solved by MinRes
// preconditioned by P = diag(|b2|, |b1|) (x) (K_x + (alpha + sqrt|b1 b2|) M_x).
// All slabs and pairs of a level iterate together, one MinRes per (slab,
// pair) with its own scalars; the vectors keep the slab layout
// [slab][time row][space], a pair occupying rows 2k, 2k+1 of its slab.
#include <cmath>

#include "kernels_common.hpp"

namespace sth {

namespace {

constexpr int kMrThreads = 256;

__device__ __forceinline__ long mr_grid_stride() { return (long)gridDim.x * kMrThreads; }

long mr_blocks(long total) { return std::max(1L, std::min((total + kMrThreads - 1) / kMrThreads, 1L << 20)); }

}  // namespace

// out[s][t][x] = (epi ? out : 0) + alpha sout[t] sum_t' M[t][t'] sin[t'] in[s][t'][x]
__global__ __launch_bounds__(kMrThreads) void k_time_mix(const double* __restrict__ in, double* __restrict__ out,
                                                          TimeRowMix m, long ns, int nt, long nx, int epi,
                                                          double alpha) {
    const long total = ns * nx;
    for (long g = (long)blockIdx.x * kMrThreads + threadIdx.x; g < total; g += mr_grid_stride()) {
        const long s = g / nx, x = g % nx;
        const double* src = in + s * nt * nx + x;
        double v[kNt];
#pragma unroll
        for (int t = 0; t < kNt; ++t) v[t] = t < nt ? m.sin[t] * src[(long)t * nx] : 0.0;
        double* dst = out + s * nt * nx + x;
        for (int t = 0; t < nt; ++t) {
            double acc = 0.0;
#pragma unroll
            for (int t2 = 0; t2 < kNt; ++t2) acc += m.M[t * kNt + t2] * v[t2];
            acc *= alpha * m.sout[t];
            dst[(long)t * nx] = epi ? dst[(long)t * nx] + acc : acc;
        }
    }
}

// q = A_bar z on the pair rows: M_x z and K_x z of each row by the tensor
// stencil of the banded 1-D matrices (M_x = M_1 (x) .. (x) M_1, K_x = sum over
// the axes of K_1 on that axis and M_1 on the others), then the 2x2 block of
// Theorem 3.10 per pair.
template <int DIM>
__global__ __launch_bounds__(kMrThreads) void k_pair_apply(const double* __restrict__ z, double* __restrict__ q,
                                                            const double* __restrict__ M1b,
                                                            const double* __restrict__ K1b, int n, int p,
                                                            long ns, int nt, PairOps ops) {
    const long nx = DIM == 3 ? (long)n * n * n : (long)n * n;
    const long total = ns * ops.npairs * nx;
    const int B = 2 * p + 1;
    for (long g = (long)blockIdx.x * kMrThreads + threadIdx.x; g < total; g += mr_grid_stride()) {
        const long x = g % nx;
        const long sk = g / nx;
        const int k = (int)(sk % ops.npairs);
        const long s = sk / ops.npairs;
        const double* za = z + (s * nt + 2 * k) * nx;
        const double* zb = za + nx;
        const int ix = (int)(x % n), iy = (int)((x / n) % n), iz = DIM == 3 ? (int)(x / ((long)n * n)) : 0;
        double ma = 0.0, ka = 0.0, mb = 0.0, kb = 0.0;
        for (int cz = 0; cz < (DIM == 3 ? B : 1); ++cz) {
            const int jz = DIM == 3 ? iz - p + cz : 0;
            if (DIM == 3 && (jz < 0 || jz >= n)) continue;
            const double mz = DIM == 3 ? M1b[iz * B + cz] : 1.0;
            const double kz = DIM == 3 ? K1b[iz * B + cz] : 0.0;
            for (int cy = 0; cy < B; ++cy) {
                const int jy = iy - p + cy;
                if (jy < 0 || jy >= n) continue;
                const double my = M1b[iy * B + cy], ky = K1b[iy * B + cy];
                const long row = ((long)jz * n + jy) * n;
                double sma = 0.0, ska = 0.0, smb = 0.0, skb = 0.0;   // x sums with M_1 and K_1
                for (int cx = 0; cx < B; ++cx) {
                    const int jx = ix - p + cx;
                    if (jx < 0 || jx >= n) continue;
                    const double mx = M1b[ix * B + cx], kx = K1b[ix * B + cx];
                    const double va = za[row + jx], vb = zb[row + jx];
                    sma += mx * va;
                    ska += kx * va;
                    smb += mx * vb;
                    skb += kx * vb;
                }
                // M z: mz my (M_1 x); K z: kz my Mx + mz ky Mx + mz my Kx
                ma += mz * my * sma;
                mb += mz * my * smb;
                ka += (kz * my + mz * ky) * sma + mz * my * ska;
                kb += (kz * my + mz * ky) * smb + mz * my * skb;
            }
        }
        double* qa = q + (s * nt + 2 * k) * nx;
        qa[x] = ops.a11[k] * (ka + ops.alpha[k] * ma) + ops.a12[k] * mb;
        qa[nx + x] = ops.a21[k] * ma + ops.a22[k] * (kb + ops.alpha[k] * mb);
    }
}

// the preconditioner in the spatial eigenbasis (between the transforms):
// t[s][r][m] *= scale[r] / (mu_m + shift[r]) for the n^d modes of each row
__global__ __launch_bounds__(kMrThreads) void k_pinv_scale(double* __restrict__ t, long ns, int nt, long nx,
                                                            int dim, const double* __restrict__ mu1, int n,
                                                            PinvRows pr) {
    const long total = ns * nt * nx;
    for (long g = (long)blockIdx.x * kMrThreads + threadIdx.x; g < total; g += mr_grid_stride()) {
        const long m = g % nx;
        const int r = (int)((g / nx) % nt);
        t[g] *= pr.scale[r] / (mode_shift(dim, mu1, n, m) + pr.shift[r]);
    }
}

// per (slab, pair) system: out[sys * stride] = sum over the pair's two rows of a b
__global__ __launch_bounds__(kMrThreads) void k_pair_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                          double* __restrict__ out, int stride, int nt, int npairs,
                                                          long nx) {
    const long sys = blockIdx.x;
    const long s = sys / npairs;
    const int k = (int)(sys % npairs);
    const long base = (s * nt + 2 * k) * nx;
    double acc = 0.0;
    for (long i = threadIdx.x; i < 2 * nx; i += kMrThreads) acc += a[base + i] * b[base + i];
    __shared__ double red[kMrThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kMrThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[sys * stride] = red[0];
}

// per-system MinRes state (kMrState doubles each): gamma_j, gamma_{j-1},
// c_{j-1}, c_{j-2}, s_{j-1}, s_{j-2}, eta, then the coefficients of the
// direction update (1/(gamma rho), zeta/rho, eps/rho, c eta) and the two
// dot products of the iteration (q.z, v.z)
enum { MR_GAM, MR_GAMP, MR_C1, MR_C2, MR_S1, MR_S2, MR_ETA, MR_CZ, MR_CW1, MR_CW2, MR_CX, MR_DQ, MR_DV };

__global__ void k_minres_init(double* __restrict__ st, long nsys) {
    const long i = (long)blockIdx.x * kMrThreads + threadIdx.x;
    if (i >= nsys) return;
    double* s = st + i * kMrState;
    const double g = sqrt(fmax(s[MR_DV], 0.0));
    s[MR_GAM] = g;
    s[MR_GAMP] = 1.0;
    s[MR_C1] = s[MR_C2] = 1.0;
    s[MR_S1] = s[MR_S2] = 0.0;
    s[MR_ETA] = g;
}

// v_{j+1} = A z~_j - delta_j v~_j - gamma_j v~_{j-1} with z~ = z / gamma_j,
// v~_j = v_j / gamma_j, v~_{j-1} = v_{j-1} / gamma_{j-1} and delta_j = (q.z) / gamma_j^2
__global__ __launch_bounds__(kMrThreads) void k_lanczos(const double* __restrict__ q, const double* __restrict__ vc,
                                                         const double* __restrict__ vp, double* __restrict__ vn,
                                                         const double* __restrict__ st, long ns, int nt,
                                                         int npairs, long nx) {
    const long total = ns * npairs * 2 * nx;
    for (long g = (long)blockIdx.x * kMrThreads + threadIdx.x; g < total; g += mr_grid_stride()) {
        const long e = g % (2 * nx);
        const long sys = g / (2 * nx);
        const long s = sys / npairs;
        const int k = (int)(sys % npairs);
        const long i = (s * nt + 2 * k) * nx + e;
        const double* S = st + sys * kMrState;
        const double gam = S[MR_GAM];
        if (!(gam > 0.0)) {
            vn[i] = 0.0;
            continue;
        }
        const double ig = 1.0 / gam;
        vn[i] = q[i] * ig - S[MR_DQ] * ig * ig * ig * vc[i] - gam / S[MR_GAMP] * vp[i];
    }
}

// the Givens rotations of the new column (gamma_j, delta_j, gamma_{j+1}) and
// the coefficients of the direction update; the state moves on one step
__global__ void k_minres_scalars(double* __restrict__ st, long nsys) {
    const long i = (long)blockIdx.x * kMrThreads + threadIdx.x;
    if (i >= nsys) return;
    double* S = st + i * kMrState;
    const double g = S[MR_GAM];
    if (!(g > 0.0)) {
        S[MR_CZ] = S[MR_CW1] = S[MR_CW2] = S[MR_CX] = 0.0;
        return;
    }
    const double gn = sqrt(fmax(S[MR_DV], 0.0));
    const double delta = S[MR_DQ] / (g * g);
    const double eps = S[MR_S2] * g;
    const double r1 = S[MR_C2] * g;
    const double zeta = S[MR_C1] * r1 + S[MR_S1] * delta;
    const double r2 = -S[MR_S1] * r1 + S[MR_C1] * delta;
    const double rho = hypot(r2, gn);
    if (!(rho > 0.0)) {
        S[MR_CZ] = S[MR_CW1] = S[MR_CW2] = S[MR_CX] = 0.0;
        S[MR_GAM] = 0.0;
        return;
    }
    const double c = r2 / rho, s = gn / rho;
    S[MR_CZ] = 1.0 / (g * rho);
    S[MR_CW1] = zeta / rho;
    S[MR_CW2] = eps / rho;
    S[MR_CX] = c * S[MR_ETA];
    S[MR_ETA] = -s * S[MR_ETA];
    S[MR_GAMP] = g;
    S[MR_GAM] = gn;
    S[MR_C2] = S[MR_C1];
    S[MR_C1] = c;
    S[MR_S2] = S[MR_S1];
    S[MR_S1] = s;
}

// w_j = (z~_j - zeta w_{j-1} - eps w_{j-2}) / rho into the buffer of w_{j-2};
// x += c eta w_j (x in the pair rows of y)
__global__ __launch_bounds__(kMrThreads) void k_minres_update(const double* __restrict__ zc,
                                                               const double* __restrict__ w1, double* __restrict__ w2,
                                                               double* __restrict__ y, const double* __restrict__ st,
                                                               long ns, int nt, int npairs, long nx) {
    const long total = ns * npairs * 2 * nx;
    for (long g = (long)blockIdx.x * kMrThreads + threadIdx.x; g < total; g += mr_grid_stride()) {
        const long e = g % (2 * nx);
        const long sys = g / (2 * nx);
        const long s = sys / npairs;
        const int k = (int)(sys % npairs);
        const long i = (s * nt + 2 * k) * nx + e;
        const double* S = st + sys * kMrState;
        const double w = S[MR_CZ] * zc[i] - S[MR_CW1] * w1[i] - S[MR_CW2] * w2[i];
        w2[i] = w;
        y[i] += S[MR_CX] * w;
    }
}

// after the first application of P^{-1} into y (all rows; the real rows hold
// their exact solution): move the pair rows to z_1 and clear them in y
// (the MinRes iterate starts from zero); w_{-1} = w_0 = 0 there
__global__ __launch_bounds__(kMrThreads) void k_pair_split(double* __restrict__ y, double* __restrict__ zc,
                                                            double* __restrict__ w1, double* __restrict__ w2,
                                                            double* __restrict__ vp, long ns, int nt, int npairs,
                                                            long nx) {
    const long total = ns * npairs * 2 * nx;
    for (long g = (long)blockIdx.x * kMrThreads + threadIdx.x; g < total; g += mr_grid_stride()) {
        const long e = g % (2 * nx);
        const long sys = g / (2 * nx);
        const long s = sys / npairs;
        const int k = (int)(sys % npairs);
        const long i = (s * nt + 2 * k) * nx + e;
        zc[i] = y[i];
        y[i] = 0.0;
        w1[i] = w2[i] = vp[i] = 0.0;
    }
}

hipError_t launch_time_mix(const double* in, double* out, const TimeRowMix& m, long ns, int nt, long nx, int epi,
                           double alpha, hipStream_t st) {
    if (ns <= 0 || nx <= 0) return hipSuccess;
    if (nt < 1 || nt > kNt) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_time_mix, dim3((unsigned)mr_blocks(ns * nx)), dim3(kMrThreads), 0, st, in, out, m, ns, nt,
                       nx, epi, alpha);
    return hipGetLastError();
}

hipError_t launch_pair_apply(int dim, const double* z, double* q, const double* M1b, const double* K1b, int n, int p,
                             long ns, int nt, const PairOps& ops, hipStream_t st) {
    if (ns <= 0 || ops.npairs <= 0) return hipSuccess;
    if (2 * ops.npairs > nt || nt > kNt || p < 1 || n < 1) return hipErrorInvalidValue;
    const long nx = (long)n * n * (dim == 3 ? n : 1);
    const long blocks = mr_blocks(ns * ops.npairs * nx);
    if (dim == 3)
        hipLaunchKernelGGL(k_pair_apply<3>, dim3((unsigned)blocks), dim3(kMrThreads), 0, st, z, q, M1b, K1b, n, p,
                           ns, nt, ops);
    else
        hipLaunchKernelGGL(k_pair_apply<2>, dim3((unsigned)blocks), dim3(kMrThreads), 0, st, z, q, M1b, K1b, n, p,
                           ns, nt, ops);
    return hipGetLastError();
}

hipError_t launch_pinv_scale(double* t, long ns, int nt, long nx, int dim, const double* mu1, int n,
                             const PinvRows& pr, hipStream_t st) {
    if (ns <= 0 || nx <= 0) return hipSuccess;
    if (nt < 1 || nt > kNt) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pinv_scale, dim3((unsigned)mr_blocks(ns * nt * nx)), dim3(kMrThreads), 0, st, t, ns, nt, nx,
                       dim, mu1, n, pr);
    return hipGetLastError();
}

hipError_t launch_pair_dot(const double* a, const double* b, double* state, int which, long ns, int nt, int npairs,
                           long nx, hipStream_t st) {
    const long nsys = ns * npairs;
    if (nsys <= 0) return hipSuccess;
    if (nsys > (1L << 31) - 1 || (which != 0 && which != 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pair_dot, dim3((unsigned)nsys), dim3(kMrThreads), 0, st, a, b,
                       state + (which == 0 ? MR_DQ : MR_DV), (int)kMrState, nt, npairs, nx);
    return hipGetLastError();
}

hipError_t launch_minres_init(double* state, long nsys, hipStream_t st) {
    if (nsys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minres_init, dim3((unsigned)((nsys + kMrThreads - 1) / kMrThreads)), dim3(kMrThreads), 0, st,
                       state, nsys);
    return hipGetLastError();
}

hipError_t launch_lanczos(const double* q, const double* vc, const double* vp, double* vn, const double* state,
                          long ns, int nt, int npairs, long nx, hipStream_t st) {
    if (ns <= 0 || npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lanczos, dim3((unsigned)mr_blocks(ns * npairs * 2 * nx)), dim3(kMrThreads), 0, st, q, vc, vp,
                       vn, state, ns, nt, npairs, nx);
    return hipGetLastError();
}

hipError_t launch_minres_scalars(double* state, long nsys, hipStream_t st) {
    if (nsys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minres_scalars, dim3((unsigned)((nsys + kMrThreads - 1) / kMrThreads)), dim3(kMrThreads), 0,
                       st, state, nsys);
    return hipGetLastError();
}

hipError_t launch_minres_update(const double* zc, const double* w1, double* w2, double* y, const double* state,
                                long ns, int nt, int npairs, long nx, hipStream_t st) {
    if (ns <= 0 || npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minres_update, dim3((unsigned)mr_blocks(ns * npairs * 2 * nx)), dim3(kMrThreads), 0, st, zc,
                       w1, w2, y, state, ns, nt, npairs, nx);
    return hipGetLastError();
}

hipError_t launch_pair_split(double* y, double* zc, double* w1, double* w2, double* vp, long ns, int nt, int npairs,
                             long nx, hipStream_t st) {
    if (ns <= 0 || npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_split, dim3((unsigned)mr_blocks(ns * npairs * 2 * nx)), dim3(kMrThreads), 0, st, y, zc,
                       w1, w2, vp, ns, nt, npairs, nx);
    return hipGetLastError();
}

}  // namespace sth
