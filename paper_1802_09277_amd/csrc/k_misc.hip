// gfx950 kernels of the space-time slab solver: fixed-order sums and the
// flags of speculative cycles, time restriction and prolongation (Section
// 3.1), the banded spatial transfers of a space-time coarsening step, fills,
// norms, the load vector and the Krylov vector operations.
#include <algorithm>

#include "kernels_common.hpp"

namespace sth {

// one block: out[0] = sum of the per-block partial sums (fixed order), also
// stored to out_host (device address of mapped, coherent pinned host
// memory) when given, which the host reads once the stream has passed
constexpr int kSumThreads = 1024;
__global__ __launch_bounds__(kSumThreads) void k_sum_partials(const double* __restrict__ partial, int count,
                                                              double* out, double* out_host, int nsum = 1,
                                                              const int* guard = nullptr,
                                                              CycleFlag flag = CycleFlag{}) {
    if (guard_off(guard)) {
        // a skipped cycle stops the cycles guarded by its own flag too
        if (flag.dev && threadIdx.x == 0) {
            *flag.dev = 0;
            if (flag.host) *flag.host = 0;
            if (flag.seq) {
                __threadfence_system();
                *flag.seq = flag.seq_val;
            }
        }
        return;
    }
    constexpr int NW = kSumThreads / 64, NA = 8;
    __shared__ double red[NW];
    __shared__ double res[3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < nsum; ++j) {
        // NA independent accumulators per thread (loads in flight together),
        // entry i going to accumulator (i / kSumThreads) % NA: a fixed order
        const double* p = partial + (long)j * count;
        double a[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q) a[q] = 0.0;
        for (int i0 = 0; i0 < count; i0 += NA * kSumThreads) {
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                const int i = i0 + q * kSumThreads + (int)threadIdx.x;
                a[q] += i < count ? p[i] : 0.0;
            }
        }
        double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < NW; ++w) t += red[w];
            out[j] = t;
            if (out_host) out_host[j] = t;
            if (j < 3) res[j] = t;
        }
        __syncthreads();
    }
    if (flag.dev && threadIdx.x == 0) {
        int go;
        if (flag.exact) {
            // the host's final test on ||r|| = sqrt(sum) against thr[1] = rtol ||f||
            const double rn = sqrt(res[0]);
            go = (!isfinite(rn) || !(rn > flag.thr[1])) ? 1 : 0;
        } else {
            const double ssq = res[0], wsq = nsum > 1 ? res[1] : 0.0;
            const double lo2 = fmax(flag.nb_lo * ssq, (1.0 - 1e-8) * wsq);
            go = (isfinite(ssq) && isfinite(wsq) && lo2 > flag.thr[0]) ? 1 : 0;
        }
        *flag.dev = go;
        if (flag.host) *flag.host = go;
        if (flag.seq) {
            __threadfence_system();
            *flag.seq = flag.seq_val;
        }
    }
}

// *flag = value (one thread)
// and optionally *thr = thr_value (negative: left as it is)
__global__ void k_set_flag(int* flag, int value, double* thr, double thr_value, double thr_lin) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *flag = value;
        if (thr && thr_value >= 0.0) {
            thr[0] = thr_value;
            thr[1] = thr_lin;
        }
    }
}

// *thr = (rtol ||f||)^2 from f2 = ||f||^2, with ||f|| taken as 1 when it is
// 0 (the same operations as the host's stopping test)
__global__ void k_spec_threshold(double* thr, const double* f2, double rtol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double fn = sqrt(f2[0]);
        if (fn == 0.0) fn = 1.0;
        const double t = rtol * fn;
        thr[0] = t * t;
        thr[1] = t;
    }
}

hipError_t launch_spec_threshold(double* thr, const double* f2, double rtol, hipStream_t st) {
    hipLaunchKernelGGL(k_spec_threshold, dim3(1), dim3(64), 0, st, thr, f2, rtol);
    return hipGetLastError();
}

hipError_t launch_set_flag(int* flag, int value, hipStream_t st, double* thr, double thr_value, double thr_lin) {
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, st, flag, value, thr, thr_value, thr_lin);
    return hipGetLastError();
}
hipError_t launch_sum_partials(const double* partial, int count, double* out, double* out_host, int nsum,
                               const int* guard, const CycleFlag& flag, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSumThreads), 0, st, partial, count, out, out_host, nsum, guard, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// time transfers
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256) void k_restrict(Transfer tr, const double* __restrict__ r,
                                                  double* __restrict__ rc, long Sc, long Nx) {
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= Sc * Nx) return;
    long m = idx / Nx, x = idx % Nx;
    const double* a = r + (2 * m) * NT * Nx + x;    // slabs 2m and 2m+1 are contiguous
    double acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = 0.0;
#pragma unroll
    for (int t = 0; t < 2 * NT; ++t) {
        double v = a[(long)t * Nx];
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[c] += tr.P[t * kNt + c] * v;
    }
    double* o = rc + m * NT * Nx + x;
#pragma unroll
    for (int c = 0; c < NT; ++c) o[(long)c * Nx] = acc[c];
}

template <int NT>
__global__ __launch_bounds__(256) void k_prolong(Transfer tr, const double* __restrict__ e,
                                                 double* __restrict__ u, long Sc, long Nx) {
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= Sc * Nx) return;
    long m = idx / Nx, x = idx % Nx;
    const double* ec = e + m * NT * Nx + x;
    double c[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) c[k] = ec[(long)k * Nx];
    double* o = u + (2 * m) * NT * Nx + x;
#pragma unroll
    for (int t = 0; t < 2 * NT; ++t) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) v += tr.P[t * kNt + k] * c[k];
        o[(long)t * Nx] += v;
    }
}

#define STH_TR_SWITCH(KER, ...)                                                        \
    switch (Nt) {                                                                      \
        case 2: hipLaunchKernelGGL(KER<2>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        case 3: hipLaunchKernelGGL(KER<3>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        case 4: hipLaunchKernelGGL(KER<4>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        case 5: hipLaunchKernelGGL(KER<5>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        case 6: hipLaunchKernelGGL(KER<6>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        case 7: hipLaunchKernelGGL(KER<7>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        case 8: hipLaunchKernelGGL(KER<8>, grid, dim3(256), 0, st, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                          \
    }

hipError_t launch_restrict(int Nt, const Transfer& tr, const double* r, double* rc, long Sc,
                           long Nx, hipStream_t st) {
    long total = Sc * Nx;
    if (total <= 0) return hipSuccess;
    dim3 grid((unsigned)((total + 255) / 256));
    STH_TR_SWITCH(k_restrict, tr, r, rc, Sc, Nx)
    return hipGetLastError();
}

hipError_t launch_prolong(int Nt, const Transfer& tr, const double* e, double* u, long Sc,
                          long Nx, hipStream_t st) {
    long total = Sc * Nx;
    if (total <= 0) return hipSuccess;
    dim3 grid((unsigned)((total + 255) / 256));
    STH_TR_SWITCH(k_prolong, tr, e, u, Sc, Nx)
    return hipGetLastError();
}

// Banded operator along one axis of a row-major tensor [outer][n_in][inner]
// (the spatial transfers between meshes of a space-time coarsening step,
// P_x^T for the restriction, P_x for the prolongation, one axis at a time):
//   out[o][i][c] = sum_{k < W} coef[i W + k] in[o][j0[i] + k][c],
// j0[i] + W <= n_in for every i (the host pads the coefficients with zeros).
__global__ __launch_bounds__(256) void k_band_axis(const double* __restrict__ in, double* __restrict__ out, long outer,
                                                   int n_in, int n_out, long inner, const int* __restrict__ j0,
                                                   const double* __restrict__ coef, int W) {
    const long total = outer * n_out * inner;
    for (long g = (long)blockIdx.x * 256 + threadIdx.x; g < total; g += (long)gridDim.x * 256) {
        const long c = g % inner;
        const long t = g / inner;
        const int i = (int)(t % n_out);
        const long o = t / n_out;
        const double* src = in + ((o * n_in + j0[i]) * inner + c);
        const double* cf = coef + (long)i * W;
        double acc = 0.0;
        for (int k = 0; k < W; ++k) acc += cf[k] * src[(long)k * inner];
        out[g] = acc;
    }
}

hipError_t launch_band_axis(const double* in, double* out, long outer, int n_in, int n_out, long inner,
                            const int* j0, const double* coef, int W, hipStream_t st) {
    if (outer <= 0 || n_out <= 0 || inner <= 0) return hipSuccess;
    if (n_in <= 0 || W <= 0 || W > n_in) return hipErrorInvalidValue;
    const long total = outer * n_out * inner;
    const long blocks = std::min<long>((total + 255) / 256, 1L << 20);
    hipLaunchKernelGGL(k_band_axis, dim3((unsigned)blocks), dim3(256), 0, st, in, out, outer, n_in, n_out, inner, j0,
                       coef, W);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
__global__ void k_set_int(int* p, int value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = value;
}

template <typename VT>
__global__ __launch_bounds__(256) void k_fill(VT* v, long len, double val, const int* skip) {
    if (skip != nullptr && skip[0] != 0) return;
    long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) v[i] = (VT)val;
}

hipError_t launch_fill(double* v, long len, double val, hipStream_t st, const int* skip, int f32) {
    if (len <= 0) return hipSuccess;
    long blocks = (len + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (f32)
        hipLaunchKernelGGL(k_fill<float>, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<float*>(v), len,
                           val, skip);
    else
        hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)blocks), dim3(256), 0, st, v, len, val, skip);
    return hipGetLastError();
}

// *flag |= 1 when some entry of v is not zero (NaN included); the caller
// clears *flag first.  One atomic per wave that saw such an entry.
__global__ __launch_bounds__(256) void k_any_nonzero(const double* __restrict__ v, long len, int* flag) {
    int nz = 0;
    const long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) nz |= !(v[i] == 0.0);
    if (__any(nz) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_any_nonzero(const double* v, long len, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, flag, 0);
    if (len > 0) {
        long blocks = (len + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_any_nonzero, dim3((unsigned)blocks), dim3(256), 0, st, v, len, flag);
    }
    return hipGetLastError();
}

__device__ inline double block_sum_256(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(256) void k_norm2_partial(const double* __restrict__ v, long len, long chunk,
                                                       double* __restrict__ partial) {
    __shared__ double sh[256];
    long beg = (long)blockIdx.x * chunk;
    long end = beg + chunk < len ? beg + chunk : len;
    // four independent sums (four loads in flight per thread), combined in a
    // fixed order; streaming loads (each entry is read once)
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    long i = beg + threadIdx.x;
    for (; i + 768 < end; i += 1024) {
        const double a0 = __builtin_nontemporal_load(v + i), a1 = __builtin_nontemporal_load(v + i + 256);
        const double a2 = __builtin_nontemporal_load(v + i + 512), a3 = __builtin_nontemporal_load(v + i + 768);
        s0 += a0 * a0;
        s1 += a1 * a1;
        s2 += a2 * a2;
        s3 += a3 * a3;
    }
    for (; i < end; i += 256) s0 += v[i] * v[i];
    double tot = block_sum_256((s0 + s1) + (s2 + s3), sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_norm2_final(const double* __restrict__ partial, double* out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < kNormBlocks; i += 256) s += partial[i];
    double tot = block_sum_256(s, sh);
    if (threadIdx.x == 0) out[0] = tot;
}

hipError_t launch_norm2(const double* v, long len, double* partial, double* out, hipStream_t st) {
    long chunk = (len + kNormBlocks - 1) / kNormBlocks;
    if (chunk < 1) chunk = 1;
    hipLaunchKernelGGL(k_norm2_partial, dim3(kNormBlocks), dim3(256), 0, st, v, len, chunk, partial);
    hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(256), 0, st, partial, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rhs(int dim, int Nt, int n, int n_modes,
                                             const double* __restrict__ Tpart,
                                             const double* __restrict__ Xpart, double* __restrict__ f,
                                             long S, long Nx) {
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    long total = S * Nt * Nx;
    if (idx >= total) return;
    long st = idx / Nx, m = idx % Nx;        // st = s*Nt + t
    int jx = (int)(m % n);
    long rest = m / n;
    int jy = (int)(rest % n);
    int jz = (int)(rest / n);
    double v = 0.0;
    for (int q = 0; q < n_modes; ++q) {
        const double* X = Xpart + (long)q * 3 * n;
        double term = Tpart[(long)q * S * Nt + st] * X[jx] * X[n + jy];
        if (dim == 3) term *= X[2 * n + jz];
        v += term;
    }
    f[idx] = v;
}

hipError_t launch_rhs(int dim, int Nt, int n, int n_modes, const double* Tpart, const double* Xpart,
                      double* f, long S, hipStream_t st) {
    long Nx = (long)n * n * (dim == 3 ? n : 1);
    long total = S * Nt * Nx;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dim, Nt, n,
                       n_modes, Tpart, Xpart, f, S, Nx);
    return hipGetLastError();
}
// ---------------------------------------------------------------------------
// Krylov support (FGMRES outer loop): k <= kMaxKrylov vectors stored one
// after the other with stride ld.
// ---------------------------------------------------------------------------
// partial[b * kMaxKrylov + i] = block b's share of <V_i, w>, i < k; the
// elements of a block and the lanes of the reduction are visited in a fixed
// order, so the result does not depend on timing
__global__ __launch_bounds__(256) void k_multidot(const double* __restrict__ V, long ld, int k,
                                                  const double* __restrict__ w, long len,
                                                  double* __restrict__ partial) {
    double acc[kMaxKrylov];
#pragma unroll
    for (int i = 0; i < kMaxKrylov; ++i) acc[i] = 0.0;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < len; e += (long)gridDim.x * 256) {
        const double we = w[e];
#pragma unroll
        for (int i = 0; i < kMaxKrylov; ++i)
            if (i < k) acc[i] += V[i * ld + e] * we;
    }
    __shared__ double red[4][kMaxKrylov];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kMaxKrylov; ++i) {
        if (i < k) {
            double v = acc[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave][i] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < k)
        partial[(long)blockIdx.x * kMaxKrylov + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ __launch_bounds__(64) void k_multidot_final(const double* __restrict__ partial, int blocks, int k,
                                                       double* __restrict__ out) {
    const int i = threadIdx.x;
    if (i >= k) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partial[(long)b * kMaxKrylov + i];
    out[i] = s;
}

// w[e] = alpha w[e] + sum_{i<k} c[i] V_i[e]  (c on the device)
__global__ __launch_bounds__(256) void k_multiaxpy(const double* __restrict__ V, long ld, int k,
                                                   const double* __restrict__ c, double alpha,
                                                   double* __restrict__ w, long len) {
    __shared__ double cs[kMaxKrylov];
    if ((int)threadIdx.x < k) cs[threadIdx.x] = c[threadIdx.x];
    __syncthreads();
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < len; e += (long)gridDim.x * 256) {
        double v = alpha * w[e];
        for (int i = 0; i < k; ++i) v += cs[i] * V[i * ld + e];
        w[e] = v;
    }
}

static const int kKrylovBlocks = 1024;

hipError_t launch_multidot(const double* V, long ld, int k, const double* w, long len, double* partial, double* out,
                           hipStream_t st) {
    if (k < 1 || k > kMaxKrylov || len <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_multidot, dim3(kKrylovBlocks), dim3(256), 0, st, V, ld, k, w, len, partial);
    hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(64), 0, st, partial, kKrylovBlocks, k, out);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(const double* V, long ld, int k, const double* c, double alpha, double* w, long len,
                            hipStream_t st) {
    if (k < 0 || k > kMaxKrylov || len <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_multiaxpy, dim3(kKrylovBlocks), dim3(256), 0, st, V, ld, k, c, alpha, w, len);
    return hipGetLastError();
}

}  // namespace sth
