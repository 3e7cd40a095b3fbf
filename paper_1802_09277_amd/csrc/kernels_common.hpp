// Device helpers shared by the kernel translation units of the slab solver
// (guards, MFMA operand layouts, LDS tile placement, BF16 splitting, the
// per-mode shifted slab solve and the pointwise eigenbasis residual).
#pragma once
#include "kernels.hpp"

namespace sth {

// Launches of a speculatively enqueued multigrid cycle carry a guard: the
// cycle before it stored 0 there when it may have converged, and then every
// kernel of the cycle returns at once (uniformly per block, before any
// barrier), leaving all buffers untouched.
// (a uniform read: one scalar load per wave; the flag was stored by an
// earlier kernel, so the caches are current at this kernel's start)
__device__ __forceinline__ bool guard_off(const int* __restrict__ guard) {
    return guard != nullptr && guard[0] == 0;
}


typedef double d4 __attribute__((ext_vector_type(4)));

typedef float f4 __attribute__((ext_vector_type(4)));

template <typename CT> struct Mfma16;
template <> struct Mfma16<double> {
    typedef d4 acc_t;
    // D[i][j] of lane l, register r: i = l/16 + 4r, j = l%16
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma16<float> {
    typedef f4 acc_t;
    // D[i][j] of lane l, register r: i = 4(l/16) + r, j = l%16
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Grid of a persistent image loop: as many 512-thread blocks as fit on the
// 256 compute units at once (LDS-limited), at most one per image.
static long persistent_blocks(size_t shm, long nimg) {
    long per_cu = shm > 0 ? (long)((160 * 1024) / shm) : 4;
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;                 // 4 x 512 threads = 32 waves per CU
    long blocks = 256 * per_cu;
    return nimg < blocks ? nimg : blocks;
}

// The 2-D kernels below may leave the last rows and columns of an image to
// FP64 dot products (one per thread) instead of a further row and column of
// MFMA tiles; not for NT16 = 6, which has no registers left for them.
template <int NT16> constexpr bool kXform2dEdge = NT16 > 1 && NT16 < 6;

// LDS placement of an NP x NP tile (NP = 16 NT16).  FP64: rows of NP words,
// the column index XOR-ed with the low four bits of the row (and, for an even
// NT16, bit four with the row parity), so that the MFMA operand reads along a
// row (16 rows x 2 columns per half-wave) and along a column (2 rows x 16
// columns) fall into distinct banks.  FP32: rows padded to NP + 1 words.
template <typename CT, int NT16> struct TileLds {
    static constexpr int NP = NT16 * 16;
    static constexpr int SIZE = sizeof(CT) == 8 ? NP * NP : NP * (NP + 1);
    static __device__ __forceinline__ int at(int r, int c) {
        if constexpr (sizeof(CT) == 8) {
            const int s = (r & 15) | ((NT16 % 2 == 0) ? (r & 1) << 4 : 0);
            return r * NP + (c ^ s);
        } else {
            return r * (NP + 1) + c;
        }
    }
};

// Entries of an image outside its MFMA core (the last n - c0 rows, then the
// last n - c0 columns of the first c0 rows) assigned to groups of g threads
// (g = 4, 2 or 1 by their count); member `part` of a group sums the k-chunks
// of 4 with index = part (mod g).  Returns false for threads without one.
__device__ __forceinline__ bool xform2d_edge(int tid, int n, int c0, int& g, int& part, int& ei, int& ej) {
    const int tail = n - c0, ne = n * n - c0 * c0;
    g = ne <= 128 ? 4 : (ne <= 256 ? 2 : 1);
    part = tid % g;
    const int e = tid / g;
    ei = -1;
    ej = 0;
    if (tail <= 0 || e >= ne) return false;
    if (e < tail * n) {
        ei = c0 + e / n;
        ej = e % n;
    } else {
        const int t = e - tail * n;
        ej = c0 + t / c0;
        ei = t % c0;
    }
    return true;
}

// sum over the g members of an edge group (adjacent lanes); all lanes call it
__device__ __forceinline__ double xform2d_edge_sum(double v, int g) {
    if (g >= 2) v += __shfl_xor(v, 1);
    if (g >= 4) v += __shfl_xor(v, 2);
    return v;
}

// k loop of the LDS-resident 2-D kernels over [0, kpad) in steps of 4 H
// (kpad a multiple of 4 H, LDS zero from n on).  With DB the operands of the
// next step are read into the second buffer before the MFMAs of the current
// one; the read is always issued (at a clamped, in-range k) so that only the
// MFMAs are conditional and the LDS counter waits stay exact.
template <int H, bool DB, typename B, typename LD, typename MM>
__device__ __forceinline__ void mfma_kloop(int kpad, LD&& ld, MM&& mma) {
    constexpr int STEP = 4 * H;
    if constexpr (DB) {
        B x, y;
        ld(0, x);
        for (int k0 = 0; k0 < kpad; k0 += 2 * STEP) {
            ld(min(k0 + STEP, kpad - STEP), y);
            mma(x);
            ld(min(k0 + 2 * STEP, kpad - STEP), x);
            if (k0 + STEP < kpad) mma(y);
        }
    } else {
        for (int k0 = 0; k0 < kpad; k0 += STEP) {
            B x;
            ld(k0, x);
            mma(x);
        }
    }
}

// MFMA tiles per axis for an n x n image stored in NT16 x NT16 tiles: all of
// them, or one fewer when the n^2 - (16 (NT16 - 1))^2 entries outside the
// smaller core fit one per thread of a 512-thread block
template <int NT16> static int xform2d_core_tiles(int n) {
    const int c0 = 16 * (NT16 - 1);
    return (kXform2dEdge<NT16> && n * n - c0 * c0 <= 512) ? NT16 - 1 : NT16;
}

// ---------------------------------------------------------------------------
// BF16x3 variant: every operand x is split into x_hi = bf16(x) and
// x_lo = bf16(x - x_hi); a product is accumulated in FP32 from the three
// MFMA bf16 products hi*hi + hi*lo + lo*hi (the lo*lo term is below the
// FP32 accumulation error).  out = M (In M^T) per image, with M = U^T for
// the forward and M = U for the inverse transform, so one matrix serves
// both products.  MFMA f32 16x16x16 bf16: lane l supplies A[l%16][4(l/16)+e]
// and B[4(l/16)+e][l%16] (e = 0..3, one 8-byte LDS read each when A is
// stored [i][k] and B as [j][k]); D[4(l/16)+r][l%16] in register r.
// ---------------------------------------------------------------------------
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);            // round to nearest even
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ void split_bf16(double v, unsigned short* hi, unsigned short* lo) {
    float x = (float)v;
    unsigned short h = to_bf16(x);
    *hi = h;
    *lo = to_bf16(x - from_bf16(h));
}

// ---------------------------------------------------------------------------
// temporal transform and shifted divide
// ---------------------------------------------------------------------------
// Reciprocals of the shifted diagonal blocks of one spatial mode, formed
// once per mode so that each slab solve of the mode is free of divisions.
// Eigen form: 1/det(Z_j + mu I) of the fixed 2x2 block j in slot 2j, and
// 1/(Z_kk + mu) of a trailing 1x1 block.  Schur form: 1/(R_kk + mu) for a
// 1x1 block, 1/det of the shifted 2x2 block in the slot of its second row.
template <int NT>
struct ModeShift {
    double mu;
    double rinv[NT];
};

template <int NT, bool SCHUR>
__device__ __forceinline__ ModeShift<NT> mode_shift_inv(const TimeMix& tm, double mu) {
    ModeShift<NT> s;
    s.mu = mu;
    if (SCHUR) {
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            double d = 1.0;
            if (tm.kind[k] == 0) {
                d = tm.R[k * kNt + k] + mu;
            } else if (tm.kind[k] == 2 && k >= 1) {
                const double a = tm.R[(k - 1) * kNt + k - 1] + mu, b = tm.R[(k - 1) * kNt + k];
                const double c = tm.R[k * kNt + k - 1], e = tm.R[k * kNt + k] + mu;
                d = a * e - b * c;
            }
            s.rinv[k] = 1.0 / d;
        }
    } else {
#pragma unroll
        for (int k = 0; k + 1 < NT; k += 2) {
            const double det = (tm.zd[k] + mu) * (tm.zd[k + 1] + mu) - tm.zo[k] * tm.zo[k + 1];
            s.rinv[k] = 1.0 / det;
            s.rinv[k + 1] = 0.0;
        }
        if (NT % 2) s.rinv[NT - 1] = 1.0 / (tm.zd[NT - 1] + mu);
    }
    return s;
}

// z = A_m^{-1} g for one slab and spatial mode: h = W g, the shifted block
// diagonal (eigen form) or quasi-triangular (Schur form) system, z = V y.
template <int NT, bool SCHUR>
__device__ __forceinline__ void shifted_solve(const TimeMix& tm, const ModeShift<NT>& sh, const double* g,
                                              double* z) {
    const double mu = sh.mu;
    double h[NT], y[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) h[t] = 0.0;
#pragma unroll
    for (int t2 = 0; t2 < NT; ++t2) {
#pragma unroll
        for (int t = 0; t < NT; ++t) h[t] += tm.W[t * kNt + t2] * g[t2];
    }
    if (SCHUR) {
        // (R + mu I) y = h, R quasi upper triangular: back substitution over
        // its 1x1 and 2x2 diagonal blocks
#pragma unroll
        for (int k = NT - 1; k >= 0; --k) {
            if (tm.kind[k] == 1) continue;                       // solved with its second row
            if (tm.kind[k] == 0) {
                double r = h[k];
#pragma unroll
                for (int j = k + 1; j < NT; ++j) r -= tm.R[k * kNt + j] * y[j];
                y[k] = r * sh.rinv[k];
            } else if (k >= 1) {                                 // rows k-1, k
                double r0 = h[k - 1], r1 = h[k];
#pragma unroll
                for (int j = k + 1; j < NT; ++j) {
                    r0 -= tm.R[(k - 1) * kNt + j] * y[j];
                    r1 -= tm.R[k * kNt + j] * y[j];
                }
                const double a = tm.R[(k - 1) * kNt + k - 1] + mu, b = tm.R[(k - 1) * kNt + k];
                const double c = tm.R[k * kNt + k - 1], d = tm.R[k * kNt + k] + mu;
                y[k - 1] = (d * r0 - b * r1) * sh.rinv[k];
                y[k] = (a * r1 - c * r0) * sh.rinv[k];
            }
        }
    } else {
        // fixed 2x2 blocks: [[p + mu, q], [r, s + mu]]^{-1} = [[s + mu, -q], [-r, p + mu]] / det
#pragma unroll
        for (int k = 0; k + 1 < NT; k += 2) {
            y[k] = ((tm.zd[k + 1] + mu) * h[k] - tm.zo[k] * h[k + 1]) * sh.rinv[k];
            y[k + 1] = ((tm.zd[k] + mu) * h[k + 1] - tm.zo[k + 1] * h[k]) * sh.rinv[k];
        }
        if (NT % 2) y[NT - 1] = h[NT - 1] * sh.rinv[NT - 1];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) v += tm.V[t * kNt + k] * y[k];
        z[t] = v;
    }
}

// one solve for a mode: the reciprocals are formed on the spot
template <int NT, bool SCHUR>
__device__ __forceinline__ void shifted_solve(const TimeMix& tm, double mu, const double* g, double* z) {
    shifted_solve<NT, SCHUR>(tm, mode_shift_inv<NT, SCHUR>(tm, mu), g, z);
}

__device__ __forceinline__ double mode_shift(int dim, const double* mu1, int n, long m) {
    int jx = (int)(m % n);
    long rest = m / n;
    int jy = (int)(rest % n);
    // in 2-D the z entry is read but not used: rest / n is 0 for the n^2 modes
    // and small for the zero-padded modes past them (clamped to the table)
    const double muz = mu1[min(rest / n, (long)n - 1)];
    double mu = mu1[jx] + mu1[jy];
    return dim == 3 ? mu + muz : mu;
}


// Weights of a spatial mode in the two-sided bounds of the B-spline residual
// norm (vw: per axis and 1-D mode, the diagonal entry d and the absolute row
// sum a of G = C^T C): lower v = 2 prod d - prod a, upper w = prod a over the
// axes, so that sum_m v_m r^_m^2 <= ||r||^2 <= sum_m w_m r^_m^2
struct ModeWeights {
    double lo, up;
};
__device__ __forceinline__ ModeWeights mode_weights(int dim, const double* __restrict__ vw, int n, long m) {
    const int jx = (int)(m % n);
    const long rest = m / n;
    const int jy = (int)(rest % n);
    // the z entries are read in 2-D too (there rest / n = 0, or small past
    // the n^2 modes in the zero padding, clamped to the table), so that every
    // load goes out at once; multiplying by 1 leaves the 2-D value exact
    const int jz = (int)min(rest / n, (long)n - 1);
    const double dz = vw[2 * jz], az = vw[2 * jz + 1];
    double d = vw[2 * jx] * vw[2 * jy], a = vw[2 * jx + 1] * vw[2 * jy + 1];
    d *= dim == 3 ? dz : 1.0;
    a *= dim == 3 ? az : 1.0;
    return ModeWeights{2.0 * d - a, a};
}

// block sums of three per-thread values into partial[b], partial[nb + b]
// and partial[2 nb + b] (nb blocks; fixed order)
__device__ __forceinline__ void block_sum3(double x, double y, double z, double* __restrict__ partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off);
        y += __shfl_xor(y, off);
        z += __shfl_xor(z, off);
    }
    __shared__ double red[12];
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = x;
        red[4 + (threadIdx.x >> 6)] = y;
        red[8 + (threadIdx.x >> 6)] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        partial[gridDim.x + blockIdx.x] = (red[4] + red[5]) + (red[6] + red[7]);
        partial[2 * gridDim.x + blockIdx.x] = (red[8] + red[9]) + (red[10] + red[11]);
    }
}

template <int NT>
__device__ __forceinline__ void eig_residual_point(const double* __restrict__ ktmt, double mu, const double* u,
                                                   double prevlast, double* g) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double a = 0.0;
#pragma unroll
        for (int t2 = 0; t2 < NT; ++t2) a += (ktmt[t * kNt + t2] + mu * ktmt[kNt * kNt + t * kNt + t2]) * u[t2];
        g[t] -= a;
    }
    g[0] += prevlast;
}

// change of the coupling value (last time row of the previous slab) made by
// a smoothing step
__device__ __forceinline__ double up_prev_delta(double prev_new, double prev_old) { return prev_new - prev_old; }

template <int NT>
__device__ __forceinline__ void prolong_add(const Transfer& tr, int h, const double* c, double* u) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) v += tr.P[(h * NT + t) * kNt + k] * c[k];
        u[t] += v;
    }
}

// one block sums the per-block partials of `nsum` sums (fixed order) into
// out[0..nsum-1] (and out_host); with a CycleFlag it also sets the
// continuation flag of a speculative cycle (launch of k_sum_partials)
hipError_t launch_sum_partials(const double* partial, int count, double* out, double* out_host, int nsum,
                               const int* guard, const CycleFlag& flag, hipStream_t st);

// Per-axis transforms with the transform matrix in LDS (np <= 256, a
// multiple of 32), the same operations as launch_xform_x / launch_xform_s.
// sym 1 and 2 (n = np = 128 or 256: xform_panel_split_supported(n)) take a
// T whose columns (forward, sym 1: T = U) or rows (inverse, sym 2: T = U^T)
// [0, n/2) are even and [n/2, n) odd under the reflection i -> n-1-i, and
// compute the same result with half the multiply-adds: the forward transform
// reads only rows k < n/2 of T, the inverse only columns j < n/2.
bool xform_panel_supported(int np);
bool xform_panel_split_supported(int n);
hipError_t launch_xform_panel_x(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                                long lines, double alpha, hipStream_t st, const int* guard, int sym = 0);
hipError_t launch_xform_panel_s(int prec, const double* in, double* out, const double* T, int n, int np, long nbatch,
                                long inner, hipStream_t st, const int* guard, int io_f32 = 0, int sym = 0);

}  // namespace sth
