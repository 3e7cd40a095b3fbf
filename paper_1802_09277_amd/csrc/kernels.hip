// gfx950 kernels of the space-time slab solver.
//
//  * k_residual  : r_n = f_n - A_n u_n + B_n u_{n-1} (eq. equ_linear_system,
//                  A_n = K_t (x) M_x + M_t (x) K_x, B_n = N_t (x) M_x with
//                  N_t = e_1 e_{N_t}^T, eq. structureAn) by sum factorisation:
//                  banded 1-D passes of M_1/K_1 through LDS per time row,
//                  then the dense N_t x N_t contraction in registers.
//  * k_xform_x / k_xform_s : the spatial eigenbasis transforms of the slab
//                  inverse (eq. equ:ST:generalDecompA with fast
//                  diagonalisation of K_x + lambda M_x) as FP64 MFMA GEMMs
//                  (v_mfma_f64_16x16x4), contiguous or strided axis.
//  * k_timemix   : per spatial mode, W, the shifted 1x1 / 2x2 divide by
//                  (Z + mu I), and V (Section 3.3 in real block form).
//  * k_restrict / k_prolong : time transfers between two fine slabs and one
//                  coarse slab (Section 3.1).
//  * k_norm2_*   : fixed-order two-stage sum of squares.
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

// ---------------------------------------------------------------------------
// residual
// ---------------------------------------------------------------------------
template <int DIM> struct ResTile;
template <> struct ResTile<2> { static constexpr int TX = 32, TY = 8, TZ = 1; };
template <> struct ResTile<3> { static constexpr int TX = 8, TY = 8, TZ = 4; };

constexpr int kMaxP = 4;
constexpr int kBand = 2 * kMaxP + 1;

template <int DIM, int NT>
__global__ __launch_bounds__(256) void k_residual(int p, int n, const double* __restrict__ M1b,
                                                  const double* __restrict__ K1b, TimeOp op,
                                                  const double* __restrict__ f,
                                                  const double* __restrict__ u, double* __restrict__ r,
                                                  long s0, double sign, int tiles_x, int tiles_y) {
    using Tl = ResTile<DIM>;
    constexpr int TX = Tl::TX, TY = Tl::TY, TZ = Tl::TZ;
    constexpr int HXM = TX + 2 * kMaxP, HYM = TY + 2 * kMaxP, HZM = (DIM == 3) ? TZ + 2 * kMaxP : 1;
    __shared__ double Us[HZM * HYM * HXM];
    __shared__ double As[HZM * HYM * TX];
    __shared__ double Bs[HZM * HYM * TX];
    __shared__ double Cs[(DIM == 3) ? HZM * TY * TX : 1];
    __shared__ double Ds[(DIM == 3) ? HZM * TY * TX : 1];
    __shared__ double bxM[TX * kBand], bxK[TX * kBand], byM[TY * kBand], byK[TY * kBand];
    __shared__ double bzM[TZ * kBand], bzK[TZ * kBand];

    const int tid = threadIdx.x;
    const int B = 2 * p + 1;
    const int HX = TX + 2 * p, HY = TY + 2 * p, HZ = (DIM == 3) ? TZ + 2 * p : 1;
    int tile = blockIdx.x;
    const int tx = tile % tiles_x;
    tile /= tiles_x;
    const int ty = tile % tiles_y;
    const int tz = tile / tiles_y;
    const int gx0 = tx * TX, gy0 = ty * TY, gz0 = tz * TZ;
    const long s = s0 + blockIdx.y;
    long Nx = (long)n * n;
    if (DIM == 3) Nx *= n;
    const long slab_len = NT * Nx;

    // band rows of the tile
    for (int i = tid; i < TX * B; i += 256) {
        int lx = i / B, k = i % B, gx = gx0 + lx;
        bxM[lx * kBand + k] = (gx < n) ? M1b[(long)gx * B + k] : 0.0;
        bxK[lx * kBand + k] = (gx < n) ? K1b[(long)gx * B + k] : 0.0;
    }
    for (int i = tid; i < TY * B; i += 256) {
        int ly = i / B, k = i % B, gy = gy0 + ly;
        byM[ly * kBand + k] = (gy < n) ? M1b[(long)gy * B + k] : 0.0;
        byK[ly * kBand + k] = (gy < n) ? K1b[(long)gy * B + k] : 0.0;
    }
    if (DIM == 3) {
        for (int i = tid; i < TZ * B; i += 256) {
            int lz = i / B, k = i % B, gz = gz0 + lz;
            bzM[lz * kBand + k] = (gz < n) ? M1b[(long)gz * B + k] : 0.0;
            bzK[lz * kBand + k] = (gz < n) ? K1b[(long)gz * B + k] : 0.0;
        }
    }

    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int gx = gx0 + lx, gy = gy0 + ly, gz = gz0 + lz;
    const bool own = gx < n && gy < n && (DIM == 2 || gz < n);

    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;

#pragma unroll
    for (int tr = 0; tr <= NT; ++tr) {
        const double* src;
        if (tr < NT) {
            src = u + s * slab_len + (long)tr * Nx;
        } else {
            if (s == 0) break;
            src = u + (s - 1) * slab_len + (long)(NT - 1) * Nx;   // end trace of slab n-1
        }
        __syncthreads();
        for (int i = tid; i < HZ * HY * HX; i += 256) {
            int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            int x = gx0 - p + hx, y = gy0 - p + hy, z = gz0 - p + hz;
            double v = 0.0;
            if (x >= 0 && x < n && y >= 0 && y < n && (DIM == 2 || (z >= 0 && z < n))) {
                long off = (DIM == 3) ? ((long)z * n + y) * n + x : (long)y * n + x;
                v = src[off];
            }
            Us[(hz * HYM + hy) * HXM + hx] = v;
        }
        __syncthreads();
        // x pass: A = M1 u, B = K1 u along x
        for (int i = tid; i < HZ * HY * TX; i += 256) {
            int ix = i % TX, hy = (i / TX) % HY, hz = i / (TX * HY);
            const double* row = &Us[(hz * HYM + hy) * HXM + ix];
            double a = 0.0, b = 0.0;
            for (int k = 0; k < B; ++k) {
                a += bxM[ix * kBand + k] * row[k];
                b += bxK[ix * kBand + k] * row[k];
            }
            As[(hz * HYM + hy) * TX + ix] = a;
            Bs[(hz * HYM + hy) * TX + ix] = b;
        }
        __syncthreads();
        double Mu = 0.0, Ku = 0.0;
        if (DIM == 2) {
            for (int k = 0; k < B; ++k) {
                double a = As[(ly + k) * TX + lx], b = Bs[(ly + k) * TX + lx];
                Mu += byM[ly * kBand + k] * a;
                Ku += byK[ly * kBand + k] * a + byM[ly * kBand + k] * b;
            }
        } else {
            // y pass: C = M1y A, D = K1y A + M1y B
            for (int i = tid; i < HZ * TY * TX; i += 256) {
                int ix = i % TX, iy = (i / TX) % TY, hz = i / (TX * TY);
                double c = 0.0, d = 0.0;
                for (int k = 0; k < B; ++k) {
                    double a = As[(hz * HYM + iy + k) * TX + ix], b = Bs[(hz * HYM + iy + k) * TX + ix];
                    c += byM[iy * kBand + k] * a;
                    d += byK[iy * kBand + k] * a + byM[iy * kBand + k] * b;
                }
                Cs[(hz * TY + iy) * TX + ix] = c;
                Ds[(hz * TY + iy) * TX + ix] = d;
            }
            __syncthreads();
            for (int k = 0; k < B; ++k) {
                double c = Cs[((lz + k) * TY + ly) * TX + lx], d = Ds[((lz + k) * TY + ly) * TX + lx];
                Mu += bzM[lz * kBand + k] * c;
                Ku += bzK[lz * kBand + k] * c + bzM[lz * kBand + k] * d;
            }
        }
        if (tr < NT) {
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] -= op.Kt[t * kNt + tr] * Mu + op.Mt[t * kNt + tr] * Ku;
        } else {
            acc[0] += Mu;
        }
    }
    if (!own) return;
    long pt = (DIM == 3) ? ((long)gz * n + gy) * n + gx : (long)gy * n + gx;
    double* rs = r + s * slab_len + pt;
    const double* fs = f ? f + s * slab_len + pt : nullptr;
#pragma unroll
    for (int t = 0; t < NT; ++t) rs[(long)t * Nx] = (fs ? fs[(long)t * Nx] : 0.0) + sign * acc[t];
}

template <int DIM>
static hipError_t residual_dim(int Nt, int p, int n, const double* M1b, const double* K1b,
                               const TimeOp& op, const double* f, const double* u, double* r,
                               long s0, long ns, double sign, hipStream_t st) {
    using Tl = ResTile<DIM>;
    int tiles_x = (n + Tl::TX - 1) / Tl::TX, tiles_y = (n + Tl::TY - 1) / Tl::TY;
    int tiles_z = (DIM == 3) ? (n + Tl::TZ - 1) / Tl::TZ : 1;
    dim3 grid(tiles_x * tiles_y * tiles_z, (unsigned)ns);
#define STH_RES_CASE(NTV)                                                                          \
    case NTV:                                                                                      \
        hipLaunchKernelGGL((k_residual<DIM, NTV>), grid, dim3(256), 0, st, p, n, M1b, K1b, op, f, \
                           u, r, s0, sign, tiles_x, tiles_y);                                      \
        break;
    switch (Nt) {
        STH_RES_CASE(2) STH_RES_CASE(3) STH_RES_CASE(4) STH_RES_CASE(5)
        STH_RES_CASE(6) STH_RES_CASE(7) STH_RES_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef STH_RES_CASE
    return hipGetLastError();
}

// 2D residual with whole rows per block: thread column x (one per thread,
// TXT >= n threads across a row), RT thread rows, RY output rows per thread.
// Per time row of u: the (TY + 2P) x n strip is staged in LDS (x halo zero),
// the x pass (M_1, K_1 along x) goes to LDS, the y pass and the temporal
// contraction stay in registers.
constexpr int kRY = 4;

// MAXR: rows of the (TY + 2P)-row strip that one thread stages (RT = 1:
// kRY + 2P; RT >= 2: at most kRY + P)
template <int NT, int P, int MAXR>
__global__ __launch_bounds__(512) void k_residual2d(int n, int TXT, int RT, const double* __restrict__ M1b,
                                                     const double* __restrict__ K1b, const double* __restrict__ ktmt,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ u, double* __restrict__ r,
                                                     long s0, double sign) {
    constexpr int B = 2 * P + 1;
    extern __shared__ double sm[];
    const int TY = RT * kRY, HY = TY + 2 * P, W = n + 2 * P;
    double* Us = sm;
    double* As = Us + HY * W;
    double* Bs = As + HY * n;
    double* byM = Bs + HY * n;
    double* byK = byM + TY * B;
    const int nthreads = TXT * RT;
    const int tid = threadIdx.x;
    const int xr = tid % TXT, yr = tid / TXT;
    const int y0 = blockIdx.x * TY;
    const long s = s0 + blockIdx.y;
    const long Nx = (long)n * n, slab = NT * Nx;
    for (int i = tid; i < HY * 2 * P; i += nthreads) {
        int rr = i / (2 * P), c = i % (2 * P);
        Us[rr * W + (c < P ? c : n + c)] = 0.0;
    }
    for (int i = tid; i < TY * B; i += nthreads) {
        int gy = y0 + i / B;
        byM[i] = gy < n ? M1b[(long)gy * B + i % B] : 0.0;
        byK[i] = gy < n ? K1b[(long)gy * B + i % B] : 0.0;
    }
    const bool xin = xr < n;
    double bxM[B], bxK[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
        bxM[k] = xin ? M1b[(long)xr * B + k] : 0.0;
        bxK[k] = xin ? K1b[(long)xr * B + k] : 0.0;
    }
    double acc[kRY][NT];
#pragma unroll
    for (int i = 0; i < kRY; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = 0.0;

    // rows of u needed per time row: staged through registers one time row
    // ahead, so the global loads of row tr+1 overlap the LDS passes of row tr
    const int NR = (s > 0) ? NT + 1 : NT;
    double pre[MAXR];
    auto load_rows = [&](int tr) {
        const double* src = (tr < NT) ? u + s * slab + (long)tr * Nx
                                       : u + (s - 1) * slab + (long)(NT - 1) * Nx;   // end trace of slab n-1
#pragma unroll
        for (int k = 0; k < MAXR; ++k) {
            const int rr = yr + RT * k, gy = y0 - P + rr;
            pre[k] = (xin && rr < HY && gy >= 0 && gy < n) ? src[(long)gy * n + xr] : 0.0;
        }
    };
    load_rows(0);
#pragma unroll 1
    for (int tr = 0; tr < NR; ++tr) {
        // column tr of K_t and M_t: uniform loads from the device copy
        double kc[NT], mc[NT];
        const int trc = tr < NT ? tr : 0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            kc[t] = ktmt[t * kNt + trc];
            mc[t] = ktmt[kNt * kNt + t * kNt + trc];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MAXR; ++k) {
            const int rr = yr + RT * k;
            if (xin && rr < HY) Us[rr * W + P + xr] = pre[k];
        }
        if (tr + 1 < NR) load_rows(tr + 1);
        __syncthreads();
        if (xin) {
            for (int rr = yr; rr < HY; rr += RT) {
                const double* row = Us + rr * W + xr;
                double a = 0.0, b = 0.0;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    a += bxM[k] * row[k];
                    b += bxK[k] * row[k];
                }
                As[rr * n + xr] = a;
                Bs[rr * n + xr] = b;
            }
        }
        __syncthreads();
        if (xin) {
#pragma unroll
            for (int i = 0; i < kRY; ++i) {
                const int ly = yr + RT * i;
                double Mu = 0.0, Ku = 0.0;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    double a = As[(ly + k) * n + xr], b = Bs[(ly + k) * n + xr];
                    double m = byM[ly * B + k];
                    Mu += m * a;
                    Ku += byK[ly * B + k] * a + m * b;
                }
                if (tr < NT) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[i][t] -= kc[t] * Mu + mc[t] * Ku;
                } else {
                    acc[i][0] += Mu;
                }
            }
        }
    }
    if (!xin) return;
#pragma unroll
    for (int i = 0; i < kRY; ++i) {
        const int gy = y0 + yr + RT * i;
        if (gy >= n) continue;
        const long off = s * slab + (long)gy * n + xr;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            double fv = f ? f[off + (long)t * Nx] : 0.0;
            r[off + (long)t * Nx] = fv + sign * acc[i][t];
        }
    }
}

template <int NT, int P>
static hipError_t residual2d_launch(int n, const double* M1b, const double* K1b, const double* ktmt,
                                    const double* f, const double* u, double* r, long s0, long ns, double sign,
                                    hipStream_t st) {
    int TXT = (n + 7) / 8 * 8;
    int RT = TXT >= 256 ? 1 : 256 / TXT;
    int TY = RT * kRY, HY = TY + 2 * P;
    size_t shm = sizeof(double) * ((size_t)HY * (n + 2 * P) + 2 * (size_t)HY * n + 2 * (size_t)TY * (2 * P + 1));
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_residual2d<NT, P, kRY + 2 * P>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_residual2d<NT, P, kRY + P>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    dim3 grid((unsigned)((n + TY - 1) / TY), (unsigned)ns);
    if (RT == 1)
        hipLaunchKernelGGL((k_residual2d<NT, P, kRY + 2 * P>), grid, dim3(TXT * RT), shm, st, n, TXT, RT, M1b, K1b,
                           ktmt, f, u, r, s0, sign);
    else
        hipLaunchKernelGGL((k_residual2d<NT, P, kRY + P>), grid, dim3(TXT * RT), shm, st, n, TXT, RT, M1b, K1b,
                           ktmt, f, u, r, s0, sign);
    return hipGetLastError();
}

template <int P>
static hipError_t residual2d_nt(int Nt, int n, const double* M1b, const double* K1b, const double* ktmt,
                                const double* f, const double* u, double* r, long s0, long ns, double sign,
                                hipStream_t st) {
    switch (Nt) {
        case 2: if (P + 1 <= 2) return residual2d_launch<2, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st); break;
        case 3: if (P + 1 <= 3) return residual2d_launch<3, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st); break;
        case 4: if (P + 1 <= 4) return residual2d_launch<4, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st); break;
        case 5: return residual2d_launch<5, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
        case 6: return residual2d_launch<6, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
        case 7: return residual2d_launch<7, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
        case 8: return residual2d_launch<8, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
        default: break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_residual(int dim, int Nt, int p, int n, const double* M1b, const double* K1b,
                           const TimeOp& op, const double* ktmt, const double* f, const double* u, double* r,
                           long s0, long ns, double sign, hipStream_t st) {
    if (ns <= 0) return hipSuccess;
    if (p < 1 || p > kMaxP) return hipErrorInvalidValue;
    if (dim == 2) {
        int TXT = (n + 7) / 8 * 8, RT = TXT >= 256 ? 1 : 256 / TXT;
        int TY = RT * kRY, HY = TY + 2 * p;
        size_t shm = sizeof(double) * ((size_t)HY * (n + 2 * p) + 2 * (size_t)HY * n + 2 * (size_t)TY * (2 * p + 1));
        if (shm > 150 * 1024 || TXT * RT > 512) return residual_dim<2>(Nt, p, n, M1b, K1b, op, f, u, r, s0, ns, sign, st);
        switch (p) {
            case 1: return residual2d_nt<1>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
            case 2: return residual2d_nt<2>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
            case 3: return residual2d_nt<3>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
            case 4: return residual2d_nt<4>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, st);
        }
    }
    if (dim == 3) return residual_dim<3>(Nt, p, n, M1b, K1b, op, f, u, r, s0, ns, sign, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Both spatial axes of a 2-D image in one kernel: U (padded to NP x NP) and
// one image stay in LDS; every block walks over images.  DIR 0 (forward):
// out = U^T R U.  DIR 1 (inverse): Z = U Y U^T, then the epilogue EPI
// (0 store, 1 out += alpha Z, 2 out = alpha Z).  Eight waves share the
// NT16 x NT16 output tiles of each GEMM; the intermediate product goes back
// into the image buffer.  CT is the compute type: double (MFMA f64 16x16x4)
// or float (MFMA f32 16x16x4, FP32 accumulation); global data stay FP64.
// ---------------------------------------------------------------------------
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

template <typename CT, int DIR, int NT16, int EPI, bool CORE>
__global__ __launch_bounds__(512) void k_xform2d(const double* __restrict__ in, double* __restrict__ out,
                                                 const double* __restrict__ Upad, int n, long nimg,
                                                 double alpha, const int* guard, long ldi, long ldo) {
    if (guard_off(guard)) return;
    using M = Mfma16<CT>;
    using T = TileLds<CT, NT16>;
    typedef typename M::acc_t acc_t;
    constexpr int NP = NT16 * 16;
    // CORE: MFMA tiles over the first NT16 - 1 tile rows and columns only
    constexpr int NC = CORE ? NT16 - 1 : NT16;
    constexpr int TPW = (NC * NC + 7) / 8;
    // k-steps per operand buffer and double buffering, as registers allow
    constexpr int H = TPW <= 2 ? 2 : 1;
    constexpr bool DB = TPW <= 4;
    struct Buf { CT a[H][TPW], b[H][TPW]; };
    extern __shared__ double sm_raw[];
    CT* Us = reinterpret_cast<CT*>(sm_raw);   // U[k][j]
    CT* Is = Us + T::SIZE;                    // image / intermediate
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int kp = (n + 3) & ~3, kpad = (n + 4 * H - 1) / (4 * H) * (4 * H);
    // MFMA tiles cover the first c0 = 16 NC rows and columns; with CORE the
    // remaining n^2 - c0^2 <= 512 entries are FP64 dot products.  Tile slots
    // of a wave past the last tile repeat it and are not stored, so that the
    // slot loops have no branches.
    constexpr int NTILE = NC * NC, c0 = 16 * NC;
    int ti[TPW], tj[TPW];
    bool own[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tq = wave + 8 * q;
        own[q] = tq < NTILE;
        ti[q] = (own[q] ? tq : NTILE - 1) / NC;
        tj[q] = (own[q] ? tq : NTILE - 1) % NC;
    }
    int eg = 1, epart = 0, ei = -1, ej = 0;
    const bool edge = CORE && xform2d_edge(tid, n, c0, eg, epart, ei, ej);
    for (int i = tid; i < NP * NP; i += 512) Us[T::at(i / NP, i % NP)] = (CT)Upad[i];
    const long nn = (long)n * n;
    // the next image is staged in registers while the current one is in the
    // MFMA products (blocks are persistent over images)
    constexpr int PER = (NP * NP + 511) / 512;
    double pre[PER];
    auto load_img = [&](long img) {
        const double* src = in + img * ldi;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + 512 * k, r = i / NP, c = i % NP;
            pre[k] = (i < NP * NP && r < n && c < n) ? src[(long)r * n + c] : 0.0;
        }
    };
    if (blockIdx.x < nimg) load_img(blockIdx.x);
    for (long img = blockIdx.x; img < nimg; img += gridDim.x) {
        __syncthreads();
        int nz = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + 512 * k;
            if (i < NP * NP) Is[T::at(i / NP, i % NP)] = (CT)pre[k];
            nz |= pre[k] != 0.0;
        }
        if (img + gridDim.x < nimg) load_img(img + gridDim.x);
        // an image of zeros (e.g. a zero initial guess) maps to zeros
        if (!__syncthreads_or(nz)) {
            if (EPI != 1) {
                double* dst = out + img * ldo;
                for (long i = tid; i < nn; i += 512) dst[i] = 0.0;
            }
            continue;
        }
        acc_t acc[TPW];
        auto mma = [&](const Buf& x) {
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int q = 0; q < TPW; ++q) acc[q] = M::op(x.a[h][q], x.b[h][q], acc[q]);
        };
        // first product: T1 = R U (forward) or Y U^T (inverse)
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = acc_t{0, 0, 0, 0};
        mfma_kloop<H, DB, Buf>(kpad, [&](int k0, Buf& x) {
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    const int k = k0 + 4 * h + lk;
                    x.a[h][q] = Is[T::at(ti[q] * 16 + lr, k)];
                    x.b[h][q] = (DIR == 0) ? Us[T::at(k, tj[q] * 16 + lr)] : Us[T::at(tj[q] * 16 + lr, k)];
                }
        }, mma);
        // edge entries of T1 (rows and columns from n on are zero in LDS)
        double e = 0.0;
        if (edge) {
            for (int k0 = 4 * epart; k0 < kp; k0 += 4 * eg) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    e += (double)Is[T::at(ei, k0 + kk)] *
                         (double)((DIR == 0) ? Us[T::at(k0 + kk, ej)] : Us[T::at(ej, k0 + kk)]);
            }
        }
        if (CORE) e = xform2d_edge_sum(e, eg);
        __syncthreads();
        // T1 over the image (rows and columns from n on stay zero)
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (own[q]) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    Is[T::at(ti[q] * 16 + M::row(lk, rr), tj[q] * 16 + lr)] = acc[q][rr];
            }
        }
        if (edge && epart == 0) Is[T::at(ei, ej)] = (CT)e;
        __syncthreads();
        // second product: U^T T1 (forward) or U T1 (inverse)
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = acc_t{0, 0, 0, 0};
        mfma_kloop<H, DB, Buf>(kpad, [&](int k0, Buf& x) {
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    const int k = k0 + 4 * h + lk;
                    x.a[h][q] = (DIR == 0) ? Us[T::at(k, ti[q] * 16 + lr)] : Us[T::at(ti[q] * 16 + lr, k)];
                    x.b[h][q] = Is[T::at(k, tj[q] * 16 + lr)];
                }
        }, mma);
        e = 0.0;
        if (edge) {
            for (int k0 = 4 * epart; k0 < kp; k0 += 4 * eg) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    e += (double)((DIR == 0) ? Us[T::at(k0 + kk, ei)] : Us[T::at(ei, k0 + kk)]) *
                         (double)Is[T::at(k0 + kk, ej)];
            }
        }
        if (CORE) e = xform2d_edge_sum(e, eg);
        double* dst = out + img * ldo;
        auto put = [&](int i, int j, double v) {
            double* o = dst + (long)i * n + j;
            if (EPI == 0) *o = v;
            else if (EPI == 1) *o += alpha * v;
            else *o = alpha * v;
        };
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (own[q]) {
                const int j = tj[q] * 16 + lr;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int i = ti[q] * 16 + M::row(lk, rr);
                    if (i < n && j < n) put(i, j, (double)acc[q][rr]);
                }
            }
        }
        if (edge && epart == 0) put(ei, ej, e);
    }
}

// MFMA tiles per axis for an n x n image stored in NT16 x NT16 tiles: all of
// them, or one fewer when the n^2 - (16 (NT16 - 1))^2 entries outside the
// smaller core fit one per thread of a 512-thread block
template <int NT16> static int xform2d_core_tiles(int n) {
    const int c0 = 16 * (NT16 - 1);
    return (kXform2dEdge<NT16> && n * n - c0 * c0 <= 512) ? NT16 - 1 : NT16;
}

template <typename CT, int DIR, int NT16, int EPI, bool CORE>
static hipError_t xform2d_go(const double* in, double* out, const double* Upad, int n, long nimg, double alpha,
                             hipStream_t st, long* nblocks, const int* guard, long ldi, long ldo) {
    size_t shm = sizeof(CT) * 2 * (size_t)TileLds<CT, NT16>::SIZE;
    static bool attr_set = false;
    if (!attr_set) {
        // exactly the dynamic size: the block-wide vote holds a little static LDS
        hipError_t e = hipFuncSetAttribute((const void*)k_xform2d<CT, DIR, NT16, EPI, CORE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    long blocks = persistent_blocks(shm, nimg);
    if (nblocks) *nblocks = blocks;
    hipLaunchKernelGGL((k_xform2d<CT, DIR, NT16, EPI, CORE>), dim3((unsigned)blocks), dim3(512), shm, st, in, out,
                       Upad, n, nimg, alpha, guard, ldi, ldo);
    return hipGetLastError();
}

template <typename CT, int DIR, int NT16, int EPI>
static hipError_t xform2d_launch(const double* in, double* out, const double* Upad, int n, long nimg, double alpha,
                                 hipStream_t st, long* nblocks = nullptr, const int* guard = nullptr,
                                 long ldi = 0, long ldo = 0) {
    if (n > 16 * NT16 || n <= 16 * (NT16 - 1)) return hipErrorInvalidValue;
    if (ldi == 0) ldi = (long)n * n;
    if (ldo == 0) ldo = (long)n * n;
    if (ldi < (long)n * n || ldo < (long)n * n) return hipErrorInvalidValue;
    if constexpr (kXform2dEdge<NT16>) {
        if (xform2d_core_tiles<NT16>(n) < NT16)
            return xform2d_go<CT, DIR, NT16, EPI, true>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
    }
    return xform2d_go<CT, DIR, NT16, EPI, false>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
}

template <typename CT, int DIR, int EPI>
static hipError_t xform2d_np(const double* in, double* out, const double* Upad, int n, int np, long nimg,
                             double alpha, hipStream_t st, long* nblocks = nullptr, const int* guard = nullptr,
                             long ldi = 0, long ldo = 0) {
    switch (np / 16) {
        case 1: return xform2d_launch<CT, DIR, 1, EPI>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 2: return xform2d_launch<CT, DIR, 2, EPI>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 3: return xform2d_launch<CT, DIR, 3, EPI>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 4: return xform2d_launch<CT, DIR, 4, EPI>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 5: return xform2d_launch<CT, DIR, 5, EPI>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 6: return xform2d_launch<CT, DIR, 6, EPI>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        default: return hipErrorInvalidValue;
    }
}

template <typename CT>
static hipError_t xform2d_prec(int dir, int epi, const double* in, double* out, const double* Upad, int n, int np,
                               long nimg, double alpha, hipStream_t st, const int* guard, long ldi, long ldo) {
    if (dir == 0) return xform2d_np<CT, 0, 0>(in, out, Upad, n, np, nimg, 1.0, st, nullptr, guard, ldi, ldo);
    if (epi == 0) return xform2d_np<CT, 1, 0>(in, out, Upad, n, np, nimg, alpha, st, nullptr, guard, ldi, ldo);
    if (epi == 1) return xform2d_np<CT, 1, 1>(in, out, Upad, n, np, nimg, alpha, st, nullptr, guard, ldi, ldo);
    if (epi == 2) return xform2d_np<CT, 1, 2>(in, out, Upad, n, np, nimg, alpha, st, nullptr, guard, ldi, ldo);
    return hipErrorInvalidValue;
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
// Per-axis spatial transforms (any n; 3-D, and 2-D images too large for the
// LDS-resident kernel).  CT = double: MFMA f64 16x16x4; CT = float: MFMA
// f32 16x16x4 with FP32 accumulation (lane l supplies A[l%16][l/16] and
// B[l/16][l%16] in both; the result rows follow Mfma16<CT>::row).
// ---------------------------------------------------------------------------
// out[line][j] (EPI) sum_k in[line][k] T[k][j]; blocks of 64 lines x 128 columns
template <typename CT, int EPI>
__global__ __launch_bounds__(256) void k_xform_x(const double* __restrict__ in, double* __restrict__ out,
                                                 const double* __restrict__ T, int n, int np, long lines,
                                                 double alpha) {
    using M = Mfma16<CT>;
    typedef typename M::acc_t acc_t;
    // FP64: rows of 16 (in_s) and 128 (T_s) words with XOR-swizzled columns
    // (row reads of 16 rows x 2 columns and column reads of 2 rows x 16
    // columns per half-wave hit distinct banks); FP32: padded rows
    constexpr bool F64 = sizeof(CT) == 8;
    __shared__ CT in_s[F64 ? 64 * 16 : 64 * 17];
    __shared__ CT T_s[F64 ? 16 * 128 : 16 * 130];
    auto ia = [](int l, int kk) { return F64 ? l * 16 + (kk ^ (l & 15)) : l * 17 + kk; };
    auto ta = [](int kk, int jj) { return F64 ? kk * 128 + (jj ^ ((kk & 1) << 4)) : kk * 130 + jj; };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long line0 = (long)blockIdx.x * 64;
    const int j0 = blockIdx.y * 128;
    const int njt = min(8, (np - j0) / 16);
    acc_t acc[8];
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) acc[jt] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < np; k0 += 16) {
        for (int i = threadIdx.x; i < 64 * 16; i += 256) {
            int l = i >> 4, kk = i & 15;
            long line = line0 + l;
            int k = k0 + kk;
            in_s[ia(l, kk)] = (CT)((line < lines && k < n) ? in[line * n + k] : 0.0);
        }
        for (int i = threadIdx.x; i < 16 * 128; i += 256) {
            int kk = i >> 7, jj = i & 127;
            int j = j0 + jj;
            T_s[ta(kk, jj)] = (CT)((j < np) ? T[(long)(k0 + kk) * np + j] : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
            CT a = in_s[ia(wave * 16 + lr, kq * 4 + lk)];
#pragma unroll
            for (int jt = 0; jt < 8; ++jt) {
                if (jt < njt) acc[jt] = M::op(a, T_s[ta(kq * 4 + lk, jt * 16 + lr)], acc[jt]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) {
        if (jt >= njt) break;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            long line = line0 + wave * 16 + M::row(lk, rr);
            int j = j0 + jt * 16 + lr;
            if (line < lines && j < n) {
                double v = (double)acc[jt][rr];
                double* o = out + line * n + j;
                if (EPI == 0) *o = v;
                else if (EPI == 1) *o += alpha * v;
                else *o = alpha * v;
            }
        }
    }
}

// strided axis: out[b][j][i] = sum_k T[k][j] in[b][k][i]; blocks of 64 j x 64 i
template <typename CT>
__global__ __launch_bounds__(256) void k_xform_s(const double* __restrict__ in, double* __restrict__ out,
                                                 const double* __restrict__ T, int n, int np, long inner,
                                                 int nib, int njb) {
    using M = Mfma16<CT>;
    typedef typename M::acc_t acc_t;
    // FP64: rows of 64 words, bit four of the column flipped on odd rows (the
    // column reads of 2 rows x 16 columns per half-wave hit distinct banks)
    constexpr bool F64 = sizeof(CT) == 8;
    __shared__ CT in_s[F64 ? 16 * 64 : 16 * 66];
    __shared__ CT T_s[F64 ? 16 * 64 : 16 * 66];
    auto sa = [](int kk, int ii) { return F64 ? kk * 64 + (ii ^ ((kk & 1) << 4)) : kk * 66 + ii; };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    long bid = blockIdx.x;
    const int ib = (int)(bid % nib);
    bid /= nib;
    const int jb = (int)(bid % njb);
    const long b = bid / njb;
    const long i0 = (long)ib * 64;
    const int j0 = jb * 64;
    const double* inb = in + b * (long)n * inner;
    double* outb = out + b * (long)n * inner;
    const bool active = (j0 + wave * 16) < np;
    acc_t acc[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) acc[it] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < np; k0 += 16) {
        for (int i = threadIdx.x; i < 16 * 64; i += 256) {
            int kk = i >> 6, ii = i & 63;
            int k = k0 + kk;
            long ig = i0 + ii;
            in_s[sa(kk, ii)] = (CT)((k < n && ig < inner) ? inb[(long)k * inner + ig] : 0.0);
            int j = j0 + ii;
            T_s[sa(kk, ii)] = (CT)((j < np) ? T[(long)k * np + j] : 0.0);
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) {
                CT a = T_s[sa(kq * 4 + lk, wave * 16 + lr)];
#pragma unroll
                for (int it = 0; it < 4; ++it) acc[it] = M::op(a, in_s[sa(kq * 4 + lk, it * 16 + lr)], acc[it]);
            }
        }
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            int j = j0 + wave * 16 + M::row(lk, rr);
            long ig = i0 + it * 16 + lr;
            if (j < n && ig < inner) outb[(long)j * inner + ig] = (double)acc[it][rr];
        }
    }
}

// BF16x3 forms of the same two kernels: operands split into bf16 hi/lo when
// staged into LDS, three MFMA f32 16x16x16 bf16 products per k-chunk of 16
// (hi*hi + hi*lo + lo*hi), FP32 accumulation.  Both operands are stored with
// k contiguous ([row][k]) so that a lane's 4 k-values are one 8-byte read.
template <int EPI>
__global__ __launch_bounds__(256) void k_xform_x_bf16x3(const double* __restrict__ in, double* __restrict__ out,
                                                        const double* __restrict__ T, int n, int np, long lines,
                                                        double alpha) {
    __shared__ unsigned short ih[64][20], il[64][20];      // [line][k]
    __shared__ unsigned short th[128][20], tl[128][20];    // [j][k]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long line0 = (long)blockIdx.x * 64;
    const int j0 = blockIdx.y * 128;
    const int njt = min(8, (np - j0) / 16);
    f4 acc[8];
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) acc[jt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < np; k0 += 16) {
        for (int i = threadIdx.x; i < 64 * 16; i += 256) {
            int l = i >> 4, kk = i & 15;
            long line = line0 + l;
            int k = k0 + kk;
            split_bf16((line < lines && k < n) ? in[line * n + k] : 0.0, &ih[l][kk], &il[l][kk]);
        }
        for (int i = threadIdx.x; i < 16 * 128; i += 256) {
            int kk = i >> 7, jj = i & 127;
            int j = j0 + jj;
            split_bf16((j < np) ? T[(long)(k0 + kk) * np + j] : 0.0, &th[jj][kk], &tl[jj][kk]);
        }
        __syncthreads();
        const s4 ah = *reinterpret_cast<const s4*>(&ih[wave * 16 + lr][4 * lk]);
        const s4 al = *reinterpret_cast<const s4*>(&il[wave * 16 + lr][4 * lk]);
#pragma unroll
        for (int jt = 0; jt < 8; ++jt) {
            if (jt < njt) {
                const s4 bh = *reinterpret_cast<const s4*>(&th[jt * 16 + lr][4 * lk]);
                const s4 bl = *reinterpret_cast<const s4*>(&tl[jt * 16 + lr][4 * lk]);
                acc[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[jt], 0, 0, 0);
                acc[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[jt], 0, 0, 0);
                acc[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[jt], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int jt = 0; jt < 8; ++jt) {
        if (jt >= njt) break;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            long line = line0 + wave * 16 + 4 * lk + rr;
            int j = j0 + jt * 16 + lr;
            if (line < lines && j < n) {
                double v = (double)acc[jt][rr];
                double* o = out + line * n + j;
                if (EPI == 0) *o = v;
                else if (EPI == 1) *o += alpha * v;
                else *o = alpha * v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_xform_s_bf16x3(const double* __restrict__ in, double* __restrict__ out,
                                                        const double* __restrict__ T, int n, int np, long inner,
                                                        int nib, int njb) {
    __shared__ unsigned short ih[64][20], il[64][20];      // [i][k]
    __shared__ unsigned short th[64][20], tl[64][20];      // [j][k]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    long bid = blockIdx.x;
    const int ib = (int)(bid % nib);
    bid /= nib;
    const int jb = (int)(bid % njb);
    const long b = bid / njb;
    const long i0 = (long)ib * 64;
    const int j0 = jb * 64;
    const double* inb = in + b * (long)n * inner;
    double* outb = out + b * (long)n * inner;
    const bool active = (j0 + wave * 16) < np;
    f4 acc[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) acc[it] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < np; k0 += 16) {
        for (int i = threadIdx.x; i < 16 * 64; i += 256) {
            int kk = i >> 6, ii = i & 63;
            int k = k0 + kk;
            long ig = i0 + ii;
            split_bf16((k < n && ig < inner) ? inb[(long)k * inner + ig] : 0.0, &ih[ii][kk], &il[ii][kk]);
            int j = j0 + ii;
            split_bf16((j < np) ? T[(long)k * np + j] : 0.0, &th[ii][kk], &tl[ii][kk]);
        }
        __syncthreads();
        if (active) {
            // A[j][k] = T[k][j], B[k][i] = in[k][i]
            const s4 ah = *reinterpret_cast<const s4*>(&th[wave * 16 + lr][4 * lk]);
            const s4 al = *reinterpret_cast<const s4*>(&tl[wave * 16 + lr][4 * lk]);
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const s4 bh = *reinterpret_cast<const s4*>(&ih[it * 16 + lr][4 * lk]);
                const s4 bl = *reinterpret_cast<const s4*>(&il[it * 16 + lr][4 * lk]);
                acc[it] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[it], 0, 0, 0);
                acc[it] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[it], 0, 0, 0);
                acc[it] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[it], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            int j = j0 + wave * 16 + 4 * lk + rr;
            long ig = i0 + it * 16 + lr;
            if (j < n && ig < inner) outb[(long)j * inner + ig] = (double)acc[it][rr];
        }
    }
}

template <typename CT>
static void xform_x_ct(int epi, dim3 grid, hipStream_t st, const double* in, double* out, const double* T, int n,
                       int np, long lines, double alpha) {
    if (epi == 0) hipLaunchKernelGGL((k_xform_x<CT, 0>), grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha);
    else if (epi == 1) hipLaunchKernelGGL((k_xform_x<CT, 1>), grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha);
    else hipLaunchKernelGGL((k_xform_x<CT, 2>), grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha);
}

hipError_t launch_xform_x(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                          long lines, double alpha, hipStream_t st) {
    if (lines <= 0) return hipSuccess;
    if (epi < 0 || epi > 2 || prec < 0 || prec > 2) return hipErrorInvalidValue;
    dim3 grid((unsigned)((lines + 63) / 64), (unsigned)((np + 127) / 128));
    if (prec == 0) xform_x_ct<double>(epi, grid, st, in, out, T, n, np, lines, alpha);
    else if (prec == 1) xform_x_ct<float>(epi, grid, st, in, out, T, n, np, lines, alpha);
    else if (epi == 0) hipLaunchKernelGGL(k_xform_x_bf16x3<0>, grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha);
    else if (epi == 1) hipLaunchKernelGGL(k_xform_x_bf16x3<1>, grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha);
    else hipLaunchKernelGGL(k_xform_x_bf16x3<2>, grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha);
    return hipGetLastError();
}

hipError_t launch_xform_s(int prec, const double* in, double* out, const double* T, int n, int np,
                          long nbatch, long inner, hipStream_t st) {
    if (nbatch <= 0) return hipSuccess;
    if (prec < 0 || prec > 2) return hipErrorInvalidValue;
    int nib = (int)((inner + 63) / 64), njb = (np + 63) / 64;
    long blocks = nbatch * nib * njb;
    if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
    if (prec == 0)
        hipLaunchKernelGGL(k_xform_s<double>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, n, np, inner,
                           nib, njb);
    else if (prec == 1)
        hipLaunchKernelGGL(k_xform_s<float>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, n, np, inner,
                           nib, njb);
    else
        hipLaunchKernelGGL(k_xform_s_bf16x3, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, n, np, inner,
                           nib, njb);
    return hipGetLastError();
}

template <int NT16, int EPI>
__global__ __launch_bounds__(512) void k_xform2d_bf16x3(const double* __restrict__ in, double* __restrict__ out,
                                                        const double* __restrict__ Mpad, int n, long nimg,
                                                        double alpha) {
    constexpr int NP = NT16 * 16, LDB = NP + 8;     // row stride in bf16 elements (keeps 8-byte alignment)
    constexpr int NTILE = NT16 * NT16, TPW = (NTILE + 7) / 8;
    extern __shared__ double sm_raw[];
    unsigned short* Mh = reinterpret_cast<unsigned short*>(sm_raw);
    unsigned short* Ml = Mh + NP * LDB;
    unsigned short* Ih = Ml + NP * LDB;
    unsigned short* Il = Ih + NP * LDB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    for (int i = tid; i < NP * NP; i += 512) {
        int r = i / NP, c = i % NP;
        split_bf16(Mpad[i], &Mh[r * LDB + c], &Ml[r * LDB + c]);
    }
    const long nn = (long)n * n;
    constexpr int PER = (NP * NP + 511) / 512;
    double pre[PER];
    auto load_img = [&](long img) {
        const double* src = in + img * nn;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + 512 * k, r = i / NP, c = i % NP;
            pre[k] = (i < NP * NP && r < n && c < n) ? src[(long)r * n + c] : 0.0;
        }
    };
    if (blockIdx.x < nimg) load_img(blockIdx.x);
    for (long img = blockIdx.x; img < nimg; img += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + 512 * k, r = i / NP, c = i % NP;
            if (i < NP * NP) split_bf16(pre[k], &Ih[r * LDB + c], &Il[r * LDB + c]);
        }
        if (img + gridDim.x < nimg) load_img(img + gridDim.x);
        __syncthreads();
        f4 acc[TPW];
        // T1 = In M^T : A = In[i][k] (stored [i][k]), B[k][j] = M[j][k] (stored [j][k])
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < NP; k0 += 16) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const int tq = wave + 8 * q;
                if (tq < NTILE) {
                    const int ti = tq / NT16, tj = tq % NT16;
                    const int ao = (ti * 16 + lr) * LDB + k0 + 4 * lk, bo = (tj * 16 + lr) * LDB + k0 + 4 * lk;
                    s4 ah = *reinterpret_cast<const s4*>(&Ih[ao]), al = *reinterpret_cast<const s4*>(&Il[ao]);
                    s4 bh = *reinterpret_cast<const s4*>(&Mh[bo]), bl = *reinterpret_cast<const s4*>(&Ml[bo]);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();
        // T1 is the B operand of the second product: store T1[k=i][j] at [j][i]
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tq = wave + 8 * q;
            if (tq < NTILE) {
                const int ti = tq / NT16, tj = tq % NT16;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int i = ti * 16 + 4 * lk + rr, j = tj * 16 + lr;
                    split_bf16((double)acc[q][rr], &Ih[j * LDB + i], &Il[j * LDB + i]);
                }
            }
        }
        __syncthreads();
        // out = M T1 : A = M[i][k] (stored [i][k]), B = T1 (stored [j][k])
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < NP; k0 += 16) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const int tq = wave + 8 * q;
                if (tq < NTILE) {
                    const int ti = tq / NT16, tj = tq % NT16;
                    const int ao = (ti * 16 + lr) * LDB + k0 + 4 * lk, bo = (tj * 16 + lr) * LDB + k0 + 4 * lk;
                    s4 ah = *reinterpret_cast<const s4*>(&Mh[ao]), al = *reinterpret_cast<const s4*>(&Ml[ao]);
                    s4 bh = *reinterpret_cast<const s4*>(&Ih[bo]), bl = *reinterpret_cast<const s4*>(&Il[bo]);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[q], 0, 0, 0);
                }
            }
        }
        double* dst = out + img * nn;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tq = wave + 8 * q;
            if (tq < NTILE) {
                const int ti = tq / NT16, tj = tq % NT16;
                const int j = tj * 16 + lr;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int i = ti * 16 + 4 * lk + rr;
                    if (i < n && j < n) {
                        double v = (double)acc[q][rr];
                        double* o = dst + (long)i * n + j;
                        if (EPI == 0) *o = v;
                        else if (EPI == 1) *o += alpha * v;
                        else *o = alpha * v;
                    }
                }
            }
        }
    }
}

template <int NT16, int EPI>
static hipError_t xform2d_bf16_launch(const double* in, double* out, const double* Mpad, int n, long nimg,
                                      double alpha, hipStream_t st) {
    constexpr int NP = NT16 * 16;
    size_t shm = sizeof(unsigned short) * 4 * (size_t)NP * (NP + 8);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_xform2d_bf16x3<NT16, EPI>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    long blocks = persistent_blocks(shm, nimg);
    hipLaunchKernelGGL((k_xform2d_bf16x3<NT16, EPI>), dim3((unsigned)blocks), dim3(512), shm, st, in, out, Mpad,
                       n, nimg, alpha);
    return hipGetLastError();
}

template <int EPI>
static hipError_t xform2d_bf16_np(const double* in, double* out, const double* Mpad, int n, int np, long nimg,
                                  double alpha, hipStream_t st) {
    switch (np / 16) {
        case 1: return xform2d_bf16_launch<1, EPI>(in, out, Mpad, n, nimg, alpha, st);
        case 2: return xform2d_bf16_launch<2, EPI>(in, out, Mpad, n, nimg, alpha, st);
        case 3: return xform2d_bf16_launch<3, EPI>(in, out, Mpad, n, nimg, alpha, st);
        case 4: return xform2d_bf16_launch<4, EPI>(in, out, Mpad, n, nimg, alpha, st);
        case 5: return xform2d_bf16_launch<5, EPI>(in, out, Mpad, n, nimg, alpha, st);
        case 6: return xform2d_bf16_launch<6, EPI>(in, out, Mpad, n, nimg, alpha, st);
        default: return hipErrorInvalidValue;
    }
}

bool xform2d_supported(int np) { return np >= 16 && np <= kXform2dMaxNp && np % 16 == 0; }

long eig_modes(int dim, int n) {
    const long nd = (long)n * n * (dim == 3 ? n : 1);
    if (dim == 2 && xform2d_supported((n + 15) / 16 * 16)) return (nd + 15) / 16 * 16;
    return nd;
}

// Sum over nimg n x n images Y of ||C Y C^T||_F^2, written as <Y G, G Y>_F with
// G = C^T C (symmetric, padded to NP): both MFMA products read the staged
// image, there is no intermediate product to store, and one barrier pair per
// image suffices.  Per-block partial sums in a fixed order.
template <int NT16, bool CORE>
__global__ __launch_bounds__(512) void k_gram_norm2d(const double* __restrict__ in, const double* __restrict__ Gpad,
                                                     int n, long nimg, double* __restrict__ partial, long ldi) {
    using T = TileLds<double, NT16>;
    constexpr int NP = NT16 * 16;
    constexpr int NC = CORE ? NT16 - 1 : NT16;
    constexpr int TPW = (NC * NC + 7) / 8;
    constexpr int H = TPW <= 1 ? 2 : 1;
    constexpr bool DB = TPW <= 2;
    struct Buf { double o[H][4][TPW]; };
    extern __shared__ double sm_raw[];
    double* Gs = sm_raw;
    double* Ys = sm_raw + T::SIZE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int kp = (n + 3) & ~3, kpad = (n + 4 * H - 1) / (4 * H) * (4 * H);
    // MFMA tiles over the first c0 rows and columns (branch-free slots as in
    // the transform kernel), with CORE FP64 dot products for the rest
    constexpr int NTILE = NC * NC, c0 = 16 * NC;
    int ti[TPW], tj[TPW];
    bool own[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tq = wave + 8 * q;
        own[q] = tq < NTILE;
        ti[q] = (own[q] ? tq : NTILE - 1) / NC;
        tj[q] = (own[q] ? tq : NTILE - 1) % NC;
    }
    int eg = 1, epart = 0, ei = -1, ej = 0;
    const bool edge = CORE && xform2d_edge(tid, n, c0, eg, epart, ei, ej);
    for (int i = tid; i < NP * NP; i += 512) Gs[T::at(i / NP, i % NP)] = Gpad[i];
    const long nn = (long)n * n;
    constexpr int PER = (NP * NP + 511) / 512;
    double pre[PER];
    auto load_img = [&](long img) {
        const double* src = in + img * ldi;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + 512 * k, r = i / NP, c = i % NP;
            pre[k] = (i < NP * NP && r < n && c < n) ? src[(long)r * n + c] : 0.0;
        }
    };
    if (blockIdx.x < nimg) load_img(blockIdx.x);
    double ssq = 0.0;
    for (long img = blockIdx.x; img < nimg; img += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + 512 * k;
            if (i < NP * NP) Ys[T::at(i / NP, i % NP)] = pre[k];
        }
        if (img + gridDim.x < nimg) load_img(img + gridDim.x);
        __syncthreads();
        d4 a1[TPW], a2[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) a1[q] = a2[q] = d4{0.0, 0.0, 0.0, 0.0};
        mfma_kloop<H, DB, Buf>(kpad, [&](int k0, Buf& x) {
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    const int k = k0 + 4 * h + lk;
                    x.o[h][0][q] = Ys[T::at(ti[q] * 16 + lr, k)];
                    x.o[h][1][q] = Gs[T::at(k, tj[q] * 16 + lr)];
                    x.o[h][2][q] = Gs[T::at(ti[q] * 16 + lr, k)];
                    x.o[h][3][q] = Ys[T::at(k, tj[q] * 16 + lr)];
                }
        }, [&](const Buf& x) {
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    a1[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.o[h][0][q], x.o[h][1][q], a1[q], 0, 0, 0);
                    a2[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.o[h][2][q], x.o[h][3][q], a2[q], 0, 0, 0);
                }
        });
        // padded rows and columns of both products are zero
#pragma unroll
        for (int q = 0; q < TPW; ++q)
            if (own[q])
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) ssq += a1[q][rr] * a2[q][rr];
        double e1 = 0.0, e2 = 0.0;
        if (edge) {
            for (int k0 = 4 * epart; k0 < kp; k0 += 4 * eg) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    e1 += Ys[T::at(ei, k0 + kk)] * Gs[T::at(k0 + kk, ej)];
                    e2 += Gs[T::at(ei, k0 + kk)] * Ys[T::at(k0 + kk, ej)];
                }
            }
        }
        if (CORE) {
            e1 = xform2d_edge_sum(e1, eg);
            e2 = xform2d_edge_sum(e2, eg);
            if (edge && epart == 0) ssq += e1 * e2;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ssq += __shfl_xor(ssq, off);
    __syncthreads();
    double* red = sm_raw;
    if (lane == 0) red[wave] = ssq;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < 8; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// one block: out[0] = sum of the per-block partial sums (fixed order), also
// stored to out_host (device address of mapped, coherent pinned host
// memory) when given, which the host reads once the stream has passed
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int count, double* out,
                                                      double* out_host, int nsum = 1, const int* guard = nullptr,
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
    __shared__ double sh[256];
    __shared__ double res[2];
    for (int j = 0; j < nsum; ++j) {
        double s = 0.0;
        for (int i = threadIdx.x; i < count; i += 256) s += partial[(long)j * count + i];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[j] = sh[0];
            if (out_host) out_host[j] = sh[0];
            if (j < 2) res[j] = sh[0];
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

// Weight v of a spatial mode in the lower bound of the B-spline residual norm
// (vw: per axis and 1-D mode, the diagonal entry d and the absolute row sum a
// of G = C^T C; v = 2 prod d - prod a over the axes)
__device__ __forceinline__ double mode_weight(int dim, const double* __restrict__ vw, int n, long m) {
    const int jx = (int)(m % n);
    const long rest = m / n;
    const int jy = (int)(rest % n);
    // the z entries are read in 2-D too (there rest / n = 0), so that every
    // load goes out at once; multiplying by 1 leaves the 2-D value exact
    const int jz = (int)(rest / n);
    const double dz = vw[2 * jz], az = vw[2 * jz + 1];
    double d = vw[2 * jx] * vw[2 * jy], a = vw[2 * jx + 1] * vw[2 * jy + 1];
    d *= dim == 3 ? dz : 1.0;
    a *= dim == 3 ? az : 1.0;
    return 2.0 * d - a;
}

// block sums of two per-thread values into partial[b] and partial[nb + b]
__device__ __forceinline__ void block_sum2(double x, double y, double* __restrict__ partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off);
        y += __shfl_xor(y, off);
    }
    __shared__ double red[8];
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = x;
        red[4 + (threadIdx.x >> 6)] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        partial[gridDim.x + blockIdx.x] = (red[4] + red[5]) + (red[6] + red[7]);
    }
}

template <int NT16, bool CORE>
static hipError_t gram_norm2d_go(const double* in, const double* Gpad, int n, long nimg, double* partial,
                                 int max_blocks, double* out, double* out_host, hipStream_t st,
                                 const CycleFlag& flag, long ldi) {
    const size_t shm = sizeof(double) * 2 * (size_t)TileLds<double, NT16>::SIZE;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_gram_norm2d<NT16, CORE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const long blocks = persistent_blocks(shm, nimg);
    if (blocks > max_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gram_norm2d<NT16, CORE>), dim3((unsigned)blocks), dim3(512), shm, st, in, Gpad, n, nimg,
                       partial, ldi);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, (int)blocks, out, out_host, 1, nullptr,
                       flag);
    return hipGetLastError();
}

template <int NT16>
static hipError_t gram_norm2d_launch(const double* in, const double* Gpad, int n, long nimg, double* partial,
                                     int max_blocks, double* out, double* out_host, hipStream_t st,
                                     const CycleFlag& flag, long ldi) {
    if (n > 16 * NT16 || n <= 16 * (NT16 - 1)) return hipErrorInvalidValue;
    if constexpr (kXform2dEdge<NT16>) {
        if (xform2d_core_tiles<NT16>(n) < NT16)
            return gram_norm2d_go<NT16, true>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
    }
    return gram_norm2d_go<NT16, false>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
}

hipError_t launch_gram_norm2d(const double* in, const double* Gpad, int n, int np, long nimg, double* partial,
                              int max_blocks, double* out, double* out_host, hipStream_t st,
                              const CycleFlag& flag, long ldi) {
    if (nimg <= 0 || !xform2d_supported(np)) return hipErrorInvalidValue;
    if (flag.dev && !flag.thr) return hipErrorInvalidValue;
    if (ldi == 0) ldi = (long)n * n;
    if (ldi < (long)n * n) return hipErrorInvalidValue;
    switch (np / 16) {
        case 1: return gram_norm2d_launch<1>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
        case 2: return gram_norm2d_launch<2>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
        case 3: return gram_norm2d_launch<3>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
        case 4: return gram_norm2d_launch<4>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
        case 5: return gram_norm2d_launch<5>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
        case 6: return gram_norm2d_launch<6>(in, Gpad, n, nimg, partial, max_blocks, out, out_host, st, flag, ldi);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_xform2d(int prec, int dir, int epi, const double* in, double* out, const double* Upad, int n,
                          int np, long nimg, double alpha, hipStream_t st, const int* guard, long ldi, long ldo) {
    if (nimg <= 0) return hipSuccess;
    if (!xform2d_supported(np)) return hipErrorInvalidValue;
    if (prec == 0) return xform2d_prec<double>(dir, epi, in, out, Upad, n, np, nimg, alpha, st, guard, ldi, ldo);
    if (prec == 1) return xform2d_prec<float>(dir, epi, in, out, Upad, n, np, nimg, alpha, st, guard, ldi, ldo);
    return hipErrorInvalidValue;
}

hipError_t launch_xform2d_bf16x3(int epi, const double* in, double* out, const double* Mpad, int n, int np,
                                 long nimg, double alpha, hipStream_t st) {
    if (nimg <= 0) return hipSuccess;
    if (!xform2d_supported(np)) return hipErrorInvalidValue;
    if (epi == 0) return xform2d_bf16_np<0>(in, out, Mpad, n, np, nimg, 1.0, st);
    if (epi == 1) return xform2d_bf16_np<1>(in, out, Mpad, n, np, nimg, alpha, st);
    return xform2d_bf16_np<2>(in, out, Mpad, n, np, nimg, alpha, st);
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
    const double muz = mu1[rest / n];                 // in 2-D, rest / n = 0 (read, not used)
    double mu = mu1[jx] + mu1[jy];
    return dim == 3 ? mu + muz : mu;
}

template <int NT, bool SCHUR>
__global__ __launch_bounds__(256) void k_timemix(int dim, TimeMix tm, const double* __restrict__ mu1, int n,
                                                 long Nx, const double* __restrict__ in,
                                                 double* __restrict__ out, long total, const int* guard) {
    if (guard_off(guard)) return;
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    long s = idx / Nx, m = idx % Nx;
    double mu = mode_shift(dim, mu1, n, m);
    const double* gp = in + s * NT * Nx + m;
    double g[NT], z[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) g[t] = gp[(long)t * Nx];
    shifted_solve<NT, SCHUR>(tm, mu, g, z);
    double* o = out + s * NT * Nx + m;
#pragma unroll
    for (int t = 0; t < NT; ++t) o[(long)t * Nx] = z[t];
}

// Exact forward substitution over S slabs in the spatial eigenbasis, parallel
// in time.  Per mode the slab systems are A u_s = g_s + e_1 x_{s-1} with the
// scalar x_{s-1} = u_{s-1}[N_t - 1], so u_s = a_s + x_{s-1} c with
// a_s = A^{-1} g_s (independent over s) and c = A^{-1} e_1, and the scalars
// obey x_s = a_s[N_t-1] + gamma x_{s-1}, gamma = c[N_t-1].  A block holds 16
// modes (one 128-byte line per time row) x 16 slab groups: each thread solves
// its group's slabs (into out), the groups' recurrences are chained through
// LDS, and a second sweep adds x_{s-1} c.  in and out must differ.
template <int NT, bool SCHUR>
__global__ __launch_bounds__(256) void k_timemix_scan(int dim, TimeMix tm, const double* __restrict__ mu1, int n,
                                                      long Nx, const double* __restrict__ in,
                                                      double* __restrict__ out, long S, const int* guard) {
    if (guard_off(guard)) return;
    constexpr int MB = 16, G = 16, LR = 4;      // LR: slabs per group held in registers
    __shared__ double xe_s[G][MB], gl_s[G][MB];
    const int ml = threadIdx.x % MB, g = threadIdx.x / MB;
    const long m = (long)blockIdx.x * MB + ml;
    const long L = (S + G - 1) / G;
    const long sb = g * L, se = (sb + L < S) ? sb + L : S;
    const bool inreg = L <= LR;
    double c[NT], areg[LR][NT], xe = 0.0, gl = 1.0, gamma = 0.0;
    const bool active = m < Nx;
    double mu = 0.0;
    if (active) {
        mu = mode_shift(dim, mu1, n, m);
        const ModeShift<NT> sh = mode_shift_inv<NT, SCHUR>(tm, mu);
        double e1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) e1[t] = (t == 0) ? 1.0 : 0.0;
        shifted_solve<NT, SCHUR>(tm, sh, e1, c);
        gamma = c[NT - 1];
        if (inreg) {
            // all loads of the group first, then the (independent) solves
#pragma unroll
            for (int i = 0; i < LR; ++i)
                if (sb + i < se) {
                    const double* gp = in + (sb + i) * NT * Nx + m;
#pragma unroll
                    for (int t = 0; t < NT; ++t) areg[i][t] = gp[(long)t * Nx];
                }
#pragma unroll
            for (int i = 0; i < LR; ++i)
                if (sb + i < se) {
                    double a[NT];
                    shifted_solve<NT, SCHUR>(tm, sh, areg[i], a);
#pragma unroll
                    for (int t = 0; t < NT; ++t) areg[i][t] = a[t];
                    xe = a[NT - 1] + gamma * xe;  // group recurrence from x = 0
                    gl *= gamma;                  // gamma^(slabs so far)
                }
        }
        for (long s = inreg ? se : sb; s < se; ++s) {
            const double* gp = in + s * NT * Nx + m;
            double gv[NT], a[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) gv[t] = gp[(long)t * Nx];
            shifted_solve<NT, SCHUR>(tm, sh, gv, a);
            double* o = out + s * NT * Nx + m;
#pragma unroll
            for (int t = 0; t < NT; ++t) o[(long)t * Nx] = a[t];
            xe = a[NT - 1] + gamma * xe;          // group recurrence from x = 0
            gl *= gamma;                          // gamma^(slabs so far)
        }
    }
    xe_s[g][ml] = xe;
    gl_s[g][ml] = gl;
    __syncthreads();
    if (!active) return;
    double x = 0.0;                               // x entering the group
    for (int h = 0; h < g; ++h) x = xe_s[h][ml] + gl_s[h][ml] * x;
    if (inreg) {
#pragma unroll
        for (int i = 0; i < LR; ++i)
            if (sb + i < se) {
                double* o = out + (sb + i) * NT * Nx + m;
                double u[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) u[t] = areg[i][t] + x * c[t];
#pragma unroll
                for (int t = 0; t < NT; ++t) o[(long)t * Nx] = u[t];
                x = u[NT - 1];
            }
        return;
    }
    for (long s = sb; s < se; ++s) {
        double* o = out + s * NT * Nx + m;
        double u[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) u[t] = o[(long)t * Nx] + x * c[t];
#pragma unroll
        for (int t = 0; t < NT; ++t) o[(long)t * Nx] = u[t];
        x = u[NT - 1];
    }
}

hipError_t launch_timemix(int dim, int Nt, const TimeMix& tm, const double* mu1, int n, long nx,
                          const double* in, double* out, long S, bool fwdsub, hipStream_t st, const int* guard) {
    long Nx = nx > 0 ? nx : (long)n * n * (dim == 3 ? n : 1);
    long total = S * Nx;
    if (total <= 0) return hipSuccess;
    if (fwdsub && in == out) return hipErrorInvalidValue;
    dim3 grid((unsigned)((total + 255) / 256));
    dim3 gridm((unsigned)((Nx + 15) / 16));
#define STH_TM_LAUNCH(NTV, SC)                                                                           \
    if (fwdsub)                                                                                          \
        hipLaunchKernelGGL((k_timemix_scan<NTV, SC>), gridm, dim3(256), 0, st, dim, tm, mu1, n, Nx, in,   \
                           out, S, guard);                                                               \
    else                                                                                                 \
        hipLaunchKernelGGL((k_timemix<NTV, SC>), grid, dim3(256), 0, st, dim, tm, mu1, n, Nx, in, out,    \
                           total, guard);
#define STH_TM_CASE(NTV)                 \
    case NTV:                            \
        if (tm.schur) {                  \
            STH_TM_LAUNCH(NTV, true)     \
        } else {                         \
            STH_TM_LAUNCH(NTV, false)    \
        }                                \
        break;
    switch (Nt) {
        STH_TM_CASE(2) STH_TM_CASE(3) STH_TM_CASE(4) STH_TM_CASE(5)
        STH_TM_CASE(6) STH_TM_CASE(7) STH_TM_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef STH_TM_CASE
#undef STH_TM_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Iteration in the spatial eigenbasis.  With u = (I (x) U_x) u^ and
// r^ = (I (x) U_x^T) r, where U_x^T M_x U_x = I and U_x^T K_x U_x = diag(mu),
// the slab operator A_n = K_t (x) M_x + M_t (x) K_x becomes
// K_t (x) I + M_t (x) diag(mu) and B_n = N_t (x) M_x becomes N_t (x) I
// (eq. structureAn), so the residual r^_n = f^_n - A^ u^_n + B^ u^_{n-1} and
// the slab inverse are both pointwise over the spatial modes.
// ---------------------------------------------------------------------------
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

// one damped block-Jacobi step u^out = u^in + omega A^{-1}(f^ - L^ u^in); with
// zero_guess u^in is taken as 0 (and not read).  uin and uout must differ
// (the coupling reads the previous slab's old iterate).  PRO: the coarse
// correction (P_t (x) I) ec of the next coarser level is added to u^in first
// (prolongation fused into the first post-smoothing step).
template <int NT, bool PRO, bool SCHUR>
__global__ __launch_bounds__(256) void k_eig_smooth(int dim, TimeMix tm, const double* __restrict__ ktmt,
                                                    const double* __restrict__ mu1, int n, long Nx,
                                                    const double* __restrict__ fh, const double* __restrict__ uin,
                                                    double* __restrict__ uout, long total, double omega,
                                                    int zero_guess, const double* __restrict__ ec, Transfer tr,
                                                    const int* guard) {
    if (guard_off(guard)) return;
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    long s = idx / Nx, m = idx % Nx;
    double mu = mode_shift(dim, mu1, n, m);
    const long base = s * NT * Nx + m;
    double g[NT], u[NT], z[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) g[t] = fh[base + (long)t * Nx];
    if (!zero_guess) {
#pragma unroll
        for (int t = 0; t < NT; ++t) u[t] = uin[base + (long)t * Nx];
        double prev = s > 0 ? uin[base - Nx] : 0.0;          // last time row of slab s-1
        if (PRO) {
            const long mc = s / 2;
            const int h = (int)(s % 2);
            double c[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) c[k] = ec[mc * NT * Nx + m + (long)k * Nx];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                double v = 0.0;
#pragma unroll
                for (int k = 0; k < NT; ++k) v += tr.P[(h * NT + t) * kNt + k] * c[k];
                u[t] += v;
            }
            if (s > 0) {
                // last row of slab s-1: second half of coarse slab (s-1)/2
                const long mp = (s - 1) / 2;
                const int hp = (int)((s - 1) % 2);
                double v = 0.0;
#pragma unroll
                for (int k = 0; k < NT; ++k)
                    v += tr.P[(hp * NT + NT - 1) * kNt + k] * ec[mp * NT * Nx + m + (long)k * Nx];
                prev += v;
            }
        }
        eig_residual_point<NT>(ktmt, mu, u, prev, g);
    } else {
#pragma unroll
        for (int t = 0; t < NT; ++t) u[t] = 0.0;
    }
    shifted_solve<NT, SCHUR>(tm, mu, g, z);
#pragma unroll
    for (int t = 0; t < NT; ++t) uout[base + (long)t * Nx] = u[t] + omega * z[t];
}

template <int NT>
__global__ __launch_bounds__(256) void k_eig_residual(const double* __restrict__ ktmt, int dim,
                                                      const double* __restrict__ mu1, int n, long Nx,
                                                      const double* __restrict__ fh, const double* __restrict__ uh,
                                                      double* __restrict__ rh, long total) {
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    long s = idx / Nx, m = idx % Nx;
    double mu = mode_shift(dim, mu1, n, m);
    const long base = s * NT * Nx + m;
    double g[NT], u[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        g[t] = fh[base + (long)t * Nx];
        u[t] = uh[base + (long)t * Nx];
    }
    eig_residual_point<NT>(ktmt, mu, u, s > 0 ? uh[base - Nx] : 0.0, g);
#pragma unroll
    for (int t = 0; t < NT; ++t) rh[base + (long)t * Nx] = g[t];
}

// residual of slabs 2m, 2m+1 restricted to coarse slab m (P_t^T (x) I)
template <int NT>
__global__ __launch_bounds__(256) void k_eig_resid_restrict(Transfer tr, const double* __restrict__ ktmt, int dim,
                                                            const double* __restrict__ mu1, int n, long Nx,
                                                            const double* __restrict__ fh,
                                                            const double* __restrict__ uh, double* __restrict__ fc,
                                                            long total) {
    long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    long mc = idx / Nx, m = idx % Nx;
    double mu = mode_shift(dim, mu1, n, m);
    double acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const long s = 2 * mc + h;
        const long base = s * NT * Nx + m;
        double g[NT], u[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            g[t] = fh[base + (long)t * Nx];
            u[t] = uh[base + (long)t * Nx];
        }
        eig_residual_point<NT>(ktmt, mu, u, s > 0 ? uh[base - Nx] : 0.0, g);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int c = 0; c < NT; ++c) acc[c] += tr.P[(h * NT + t) * kNt + c] * g[t];
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) fc[mc * NT * Nx + m + (long)c * Nx] = acc[c];
}

// change of the coupling value (last time row of the previous slab) made by
// a smoothing step
__device__ __forceinline__ double up_prev_delta(double prev_new, double prev_old) { return prev_new - prev_old; }

// End of a cycle on the finest level, for one spatial mode and a chain of
// `chain` consecutive slabs (chain even, starting at an even slab): the
// residual r^ = f^ - L u^ of the iterate (its squares summed per block into
// partial[blockIdx.x], fixed order), the next cycle's first smoothing step
// u'^ = u^ + omega A^{-1} r^ (into uout), and the restriction of the residual
// of u'^ to the next level, fc = (P_t^T (x) I)[r'_{2k}; r'_{2k+1}].  The last
// time row of the previous slab (old and smoothed iterate) is carried in
// registers along the chain; a chain after slab 0 first repeats the
// smoothing step of its preceding slab for that row.
template <int NT, bool SCHUR>
__global__ __launch_bounds__(256) void k_eig_cycle_end(int dim, TimeMix tm, const double* __restrict__ ktmt,
                                                       const double* __restrict__ mu1, int n, long Nx,
                                                       const double* __restrict__ fh, const double* __restrict__ uin,
                                                       double* __restrict__ uout, double* __restrict__ fc,
                                                       Transfer tr, double omega, int chain, long total,
                                                       const double* __restrict__ vw,
                                                       double* __restrict__ partial) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    double ssq = 0.0, wsq = 0.0;
    if (idx < total) {
        const long q = idx / Nx, m = idx % Nx;
        const long s0 = q * chain;
        // loads first (the chain's first slab, and the slab before it), so
        // that none waits behind the per-mode setup; the next slab's f^ and
        // u^ are then loaded while the current one is processed
        double fnx[NT], unx[NT], acc[NT];
        {
            const long b = s0 * NT * Nx + m;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                fnx[t] = fh[b + (long)t * Nx];
                unx[t] = uin[b + (long)t * Nx];
            }
        }
        double pg[NT], pu[NT], pq = 0.0;
        if (s0 > 0) {
            const long b = (s0 - 1) * NT * Nx + m;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                pg[t] = fh[b + (long)t * Nx];
                pu[t] = uin[b + (long)t * Nx];
            }
            if (s0 > 1) pq = uin[b - Nx];
        }
        const double mu = mode_shift(dim, mu1, n, m);
        const ModeShift<NT> sh = mode_shift_inv<NT, SCHUR>(tm, mu);
        const double wm = mode_weight(dim, vw, n, m);
        double prev_old = 0.0, prev_new = 0.0;
        if (s0 > 0) {
            double z[NT];
            eig_residual_point<NT>(ktmt, mu, pu, pq, pg);
            shifted_solve<NT, SCHUR>(tm, sh, pg, z);
            prev_old = pu[NT - 1];
            prev_new = pu[NT - 1] + omega * z[NT - 1];
        }
#pragma unroll 1
        for (int k = 0; k < chain; ++k) {
            const int h = k & 1;
            const long b = (s0 + k) * NT * Nx + m;
            double g[NT], g2[NT], u[NT], z[NT], up[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                g[t] = fnx[t];
                u[t] = unx[t];
            }
            if (k + 1 < chain) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    fnx[t] = fh[b + NT * Nx + (long)t * Nx];
                    unx[t] = uin[b + NT * Nx + (long)t * Nx];
                }
            }
            eig_residual_point<NT>(ktmt, mu, u, prev_old, g);
            double s2 = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) s2 += g[t] * g[t];
            ssq += s2;
            wsq += wm * s2;
            shifted_solve<NT, SCHUR>(tm, sh, g, z);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                up[t] = u[t] + omega * z[t];
                uout[b + (long)t * Nx] = up[t];
            }
            // residual of u': A z = g (the block of the smoother is the slab
            // operator), so f - A u' + e_1 u'_prev = (1 - omega) g + e_1 (u'_prev - u_prev)
#pragma unroll
            for (int t = 0; t < NT; ++t) g2[t] = (1.0 - omega) * g[t];
            g2[0] += up_prev_delta(prev_new, prev_old);
            if (h == 0) {
#pragma unroll
                for (int c = 0; c < NT; ++c) acc[c] = 0.0;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int c = 0; c < NT; ++c) acc[c] += tr.P[(h * NT + t) * kNt + c] * g2[t];
            if (h == 1) {
                const long mc = (s0 + k) / 2;
#pragma unroll
                for (int c = 0; c < NT; ++c) fc[mc * NT * Nx + m + (long)c * Nx] = acc[c];
            }
            prev_old = u[NT - 1];
            prev_new = up[NT - 1];
        }
    }
    // block sums (fixed order) of ||r^||^2 and its weighted form
    block_sum2(ssq, wsq, partial);
}

// Close of a cycle on the finest level followed by the start of the next
// one, for one spatial mode and a chain of `chain` consecutive slabs (chain
// even, starting at an even slab), in one pass over f^, the pre-smoothed
// iterate u^ and the coarse correction ec:
//   u1 = u^ + (P_t (x) I) ec                       (prolongation)
//   u2 = u1 + omega A^{-1} r(u1)  -> uend          (post-smoothing step)
//   ||r(u2)||^2 summed per block into partial[blockIdx.x] (fixed order)
//   u3 = u2 + omega A^{-1} r(u2)  -> unext         (next pre-smoothing step)
//   fc = (P_t^T (x) I)[r(u3)_{2k}; r(u3)_{2k+1}]   (restriction)
// The residuals after a smoothing step follow from the identity
// r(u + omega A^{-1} g)_s = (1 - omega) g_s + e_1 (delta of the coupling row
// of slab s-1), and with it A^{-1} r(u2) = (1 - omega) A^{-1} r(u1) +
// delta A^{-1} e_1, so every slab needs one slab solve.  The coupling rows of
// the previous slab (u1, u2, u3) are carried along the chain; a chain after
// slab 0 first repeats the two steps of its two preceding slabs.
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

template <int NT, bool SCHUR>
__global__ __launch_bounds__(256) void k_eig_cycle_close(int dim, TimeMix tm, const double* __restrict__ ktmt,
                                                         const double* __restrict__ mu1, int n, long Nx,
                                                         const double* __restrict__ fh,
                                                         const double* __restrict__ upre,
                                                         const double* __restrict__ ec, double* __restrict__ uend,
                                                         double* __restrict__ unext, double* __restrict__ fc,
                                                         Transfer tr, double omega, int chain, long total,
                                                         const double* __restrict__ vw,
                                                         double* __restrict__ partial, const int* guard) {
    if (guard_off(guard)) return;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    double ssq = 0.0, wsq = 0.0;
    if (idx < total) {
        const long q = idx / Nx, m = idx % Nx;
        const long s0 = q * chain;
        const long slab = (long)NT * Nx;
        // loads first: the chain's first slab (f^, u^ and ec) and, after slab
        // 0, the two slabs before it, so that none waits behind the per-mode
        // setup below
        double fnx[NT], unx[NT], cnx[NT], c[NT], acc[NT];
        {
            const long b = s0 * slab + m, bc = (s0 / 2) * slab + m;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                fnx[t] = fh[b + (long)t * Nx];
                unx[t] = upre[b + (long)t * Nx];
                cnx[t] = ec[bc + (long)t * Nx];
            }
        }
        const long sa = s0 - 2;                 // slab s0 - 2 (even): first half of coarse slab s0/2 - 1
        double pc[NT], pua[NT], pfa[NT], pub[NT], pfb[NT], pq[NT], pqu = 0.0;
        if (s0 > 0) {
            const long ba = sa * slab + m, bc = (sa / 2) * slab + m, bb = (s0 - 1) * slab + m;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                pc[t] = ec[bc + (long)t * Nx];
                pua[t] = upre[ba + (long)t * Nx];
                pfa[t] = fh[ba + (long)t * Nx];
                pub[t] = upre[bb + (long)t * Nx];
                pfb[t] = fh[bb + (long)t * Nx];
            }
            if (sa > 0) {
                // the coupling row of slab s0 - 3 from u^ and ec
                const long bp = (sa - 1) * slab + m, bpc = ((sa - 1) / 2) * slab + m;
                pqu = upre[bp + (long)(NT - 1) * Nx];
#pragma unroll
                for (int k = 0; k < NT; ++k) pq[k] = ec[bpc + (long)k * Nx];
            }
        }
        const double mu = mode_shift(dim, mu1, n, m);
        const ModeShift<NT> sh = mode_shift_inv<NT, SCHUR>(tm, mu);
        // ca = A^{-1} e_1: a change of the coupling row moves A^{-1} r by a multiple of it
        double ca[NT];
        {
            double e1[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) e1[t] = (t == 0) ? 1.0 : 0.0;
            shifted_solve<NT, SCHUR>(tm, sh, e1, ca);
        }
        const double wm = mode_weight(dim, vw, n, m);
        // coupling rows of slab s0 - 1: u1, u2 and u3
        double p1 = 0.0, p2 = 0.0, p3 = 0.0;
        if (s0 > 0) {
            double u1[NT], g[NT], z[NT];
            double q1 = 0.0;
            if (sa > 0) {
                double v = pqu;
#pragma unroll
                for (int k = 0; k < NT; ++k) v += tr.P[(NT + NT - 1) * kNt + k] * pq[k];
                q1 = v;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                u1[t] = pua[t];
                g[t] = pfa[t];
            }
            prolong_add<NT>(tr, 0, pc, u1);
            eig_residual_point<NT>(ktmt, mu, u1, q1, g);
            shifted_solve<NT, SCHUR>(tm, sh, g, z);
            const double a1 = u1[NT - 1], a2 = u1[NT - 1] + omega * z[NT - 1];
            // slab s0 - 1 (second half of the same coarse slab): both steps
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                u1[t] = pub[t];
                g[t] = pfb[t];
            }
            prolong_add<NT>(tr, 1, pc, u1);
            eig_residual_point<NT>(ktmt, mu, u1, a1, g);
            shifted_solve<NT, SCHUR>(tm, sh, g, z);
            const double u2last = u1[NT - 1] + omega * z[NT - 1];
            const double z2last = (1.0 - omega) * z[NT - 1] + up_prev_delta(a2, a1) * ca[NT - 1];
            p1 = u1[NT - 1];
            p2 = u2last;
            p3 = u2last + omega * z2last;
        }
#pragma unroll 1
        for (int k = 0; k < chain; ++k) {
            const int h = k & 1;
            const long b = (s0 + k) * slab + m;
            double g[NT], u1[NT], u2[NT], z[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                g[t] = fnx[t];
                u1[t] = unx[t];
            }
            if (h == 0) {
#pragma unroll
                for (int t = 0; t < NT; ++t) c[t] = cnx[t];
            }
            if (k + 1 < chain) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    fnx[t] = fh[b + slab + (long)t * Nx];
                    unx[t] = upre[b + slab + (long)t * Nx];
                }
                if (h == 1) {
                    const long bc = ((s0 + k + 1) / 2) * slab + m;
#pragma unroll
                    for (int t = 0; t < NT; ++t) cnx[t] = ec[bc + (long)t * Nx];
                }
            }
            // post-smoothing step from the prolonged iterate
            prolong_add<NT>(tr, h, c, u1);
            eig_residual_point<NT>(ktmt, mu, u1, p1, g);
            shifted_solve<NT, SCHUR>(tm, sh, g, z);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                u2[t] = u1[t] + omega * z[t];
                uend[b + (long)t * Nx] = u2[t];
                g[t] *= (1.0 - omega);
            }
            const double d2 = up_prev_delta(p2, p1);
            g[0] += d2;
            // residual of the cycle's result, then the next smoothing step
            // with A^{-1} r(u2) = (1 - omega) z + d2 ca
            double s2 = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) s2 += g[t] * g[t];
            ssq += s2;
            wsq += wm * s2;
            double u3last = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double u3 = u2[t] + omega * ((1.0 - omega) * z[t] + d2 * ca[t]);
                unext[b + (long)t * Nx] = u3;
                if (t == NT - 1) u3last = u3;
                g[t] *= (1.0 - omega);
            }
            g[0] += up_prev_delta(p3, p2);
            if (h == 0) {
#pragma unroll
                for (int cc = 0; cc < NT; ++cc) acc[cc] = 0.0;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int cc = 0; cc < NT; ++cc) acc[cc] += tr.P[(h * NT + t) * kNt + cc] * g[t];
            if (h == 1) {
                const long mc = (s0 + k) / 2;
#pragma unroll
                for (int cc = 0; cc < NT; ++cc) fc[mc * slab + m + (long)cc * Nx] = acc[cc];
            }
            p1 = u1[NT - 1];
            p2 = u2[NT - 1];
            p3 = u3last;
        }
    }
    block_sum2(ssq, wsq, partial);
}

// The two coarsest levels of a V(1,1) cycle in one pass (a: second-coarsest
// level with SA slabs, b: coarsest with SA/2 slabs), from the right-hand side
// fa of level a alone:
//   u  = omega A_a^{-1} fa                       (smoothing step from zero)
//   fb = (P_t^T (x) I)(fa - L_a u) on slab pairs  ((1 - omega) fa + e_1 u_{s-1})
//   ub = L_b^{-1} fb                              (exact, parallel in time)
//   v  = u + (P_t (x) I) ub,  ua = v + omega A_a^{-1}(fa - L_a v)
// Since A_a u = omega fa, the last step needs neither fa nor a solve:
// fa - L_a v = (1 - omega) fa - A_a (P_t ub) + e_1 q with q the last time
// row of the previous slab of v, so
//   ua = (2 - omega) u + (1 - omega)(P_t (x) I) ub + omega q A_a^{-1} e_1.
// A block holds 16 modes (one 128-byte line per time row) x G slab groups of
// LA level-a and LA/2 level-b slabs per thread, kept in registers; the
// coupling rows between groups, and the recurrence of the exact solve
// (u_s = A^{-1} g_s + x_{s-1} A^{-1} e_1, x_s = a_s[N_t-1] + gamma x_{s-1}),
// pass through LDS.  Only ua is written.
template <int NT, bool SCHUR, int LAM>
__global__ __launch_bounds__(512, ((NT <= 5 && LAM <= 4) ? 4 : 2)) void k_eig_coarse_tail(int dim, const TimeMix* __restrict__ tma,
                                                         const TimeMix* __restrict__ tmb,
                                                         const double* __restrict__ mu1, int n, long Nx,
                                                         const double* __restrict__ fa, double* __restrict__ ua,
                                                         Transfer tr, double omega, int G, int LA,
                                                         const int* guard) {
    if (guard_off(guard)) return;
    constexpr int MB = 16, LBM = LAM / 2;
    __shared__ double xch[32][MB], xe_s[32][MB], gl_s[32][MB];
    const int ml = threadIdx.x % MB, g = threadIdx.x / MB;
    const long m = (long)blockIdx.x * MB + ml;
    const bool active = m < Nx;
    const int LB = LA / 2;
    const long slab = (long)NT * Nx;
    const long sa0 = (long)g * LA;                 // first level-a slab of the group (even)
    double u[LAM][NT], ub[LBM][NT];
    double mu = 0.0, ulast = 0.0;
    // (1) smoothing step from zero and restriction of its residual
    if (active) {
        mu = mode_shift(dim, mu1, n, m);
#pragma unroll
        for (int j = 0; j < LBM; ++j)
#pragma unroll
            for (int t = 0; t < NT; ++t) ub[j][t] = 0.0;
#pragma unroll
        for (int i = 0; i < LAM; ++i) {
            if (i < LA) {
                double f[NT], z[NT];
                const long b = (sa0 + i) * slab + m;
#pragma unroll
                for (int t = 0; t < NT; ++t) f[t] = fa[b + (long)t * Nx];
                shifted_solve<NT, SCHUR>(*tma, mu, f, z);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    u[i][t] = omega * z[t];
                    f[t] *= (1.0 - omega);
                }
                if (i > 0) f[0] += u[i - 1][NT - 1];
                if (i == LA - 1) ulast = u[i][NT - 1];
                const int h = i & 1;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int c = 0; c < NT; ++c) ub[i / 2][c] += tr.P[(h * NT + t) * kNt + c] * f[t];
            }
        }
        xch[g][ml] = ulast;
    }
    __syncthreads();
    if (active && g > 0) {
        // coupling row of the group's first slab: the previous group's last
        const double x0 = xch[g - 1][ml];
#pragma unroll
        for (int c = 0; c < NT; ++c) ub[0][c] += tr.P[c] * x0;     // P^T row of t = 0, h = 0
    }
    // (2) exact solve on level b, parallel in time over the groups
    double cb[NT], xe = 0.0, gl = 1.0;
    if (active) {
        double e1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) e1[t] = (t == 0) ? 1.0 : 0.0;
        shifted_solve<NT, SCHUR>(*tmb, mu, e1, cb);
        const double gamma = cb[NT - 1];
#pragma unroll
        for (int j = 0; j < LBM; ++j) {
            if (j < LB) {
                double a[NT];
                shifted_solve<NT, SCHUR>(*tmb, mu, ub[j], a);
#pragma unroll
                for (int t = 0; t < NT; ++t) ub[j][t] = a[t];
                xe = a[NT - 1] + gamma * xe;
                gl *= gamma;
            }
        }
    }
    xe_s[g][ml] = xe;
    gl_s[g][ml] = gl;
    __syncthreads();
    double vlast = 0.0;
    if (active) {
        double x = 0.0;
        for (int h = 0; h < g; ++h) x = xe_s[h][ml] + gl_s[h][ml] * x;
#pragma unroll
        for (int j = 0; j < LBM; ++j) {
            if (j < LB) {
#pragma unroll
                for (int t = 0; t < NT; ++t) ub[j][t] += x * cb[t];
                x = ub[j][NT - 1];
                if (j == LB - 1) {
                    // prolonged coupling row of the group's last level-a slab (odd)
                    vlast = ulast;
#pragma unroll
                    for (int k = 0; k < NT; ++k) vlast += tr.P[(NT + NT - 1) * kNt + k] * ub[j][k];
                }
            }
        }
    }
    __syncthreads();                               // xch is reused
    if (active) xch[g][ml] = vlast;
    __syncthreads();
    if (!active) return;
    // (3) prolongation and the post-smoothing step on level a (closed form)
    double ca[NT];
    {
        double e1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) e1[t] = (t == 0) ? 1.0 : 0.0;
        shifted_solve<NT, SCHUR>(*tma, mu, e1, ca);
    }
    double q = g > 0 ? xch[g - 1][ml] : 0.0;
#pragma unroll
    for (int i = 0; i < LAM; ++i) {
        if (i < LA) {
            const int h = i & 1;
            const long b = (sa0 + i) * slab + m;
            double pu[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                double w = 0.0;
#pragma unroll
                for (int k = 0; k < NT; ++k) w += tr.P[(h * NT + t) * kNt + k] * ub[i / 2][k];
                pu[t] = w;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
                ua[b + (long)t * Nx] = (2.0 - omega) * u[i][t] + (1.0 - omega) * pu[t] + omega * q * ca[t];
            q = u[i][NT - 1] + pu[NT - 1];
        }
    }
}

// Descent on a coarse level with a zero initial guess and one pre-smoothing
// step, for one spatial mode and a chain of `chain` slabs (chain even,
// starting at an even slab): u' = omega A^{-1} f (into uout) and the
// restriction of its residual, fc = (P_t^T (x) I)[f - L u']_{2k, 2k+1}, from one
// read of f.  The last time row of the previous slab's u' is carried along the
// chain; a chain after slab 0 first repeats the step for its preceding slab.
template <int NT, bool SCHUR>
__global__ __launch_bounds__(256) void k_eig_down(int dim, TimeMix tm, const double* __restrict__ ktmt,
                                                  const double* __restrict__ mu1, int n, long Nx,
                                                  const double* __restrict__ fl, double* __restrict__ uout,
                                                  double* __restrict__ fc, Transfer tr, double omega, int chain,
                                                  long total, const int* guard) {
    if (guard_off(guard)) return;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const long q = idx / Nx, m = idx % Nx;
    const double mu = mode_shift(dim, mu1, n, m);
    const ModeShift<NT> sh = mode_shift_inv<NT, SCHUR>(tm, mu);
    const long s0 = q * chain;
    double prev = 0.0;
    if (s0 > 0) {
        const long b = (s0 - 1) * NT * Nx + m;
        double g[NT], z[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) g[t] = fl[b + (long)t * Nx];
        shifted_solve<NT, SCHUR>(tm, sh, g, z);
        prev = omega * z[NT - 1];
    }
    double fnx[NT], acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) fnx[t] = fl[s0 * NT * Nx + m + (long)t * Nx];
#pragma unroll 1
    for (int k = 0; k < chain; ++k) {
        const int h = k & 1;
        const long b = (s0 + k) * NT * Nx + m;
        double g[NT], g2[NT], z[NT], up[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) g[t] = fnx[t];
        if (k + 1 < chain) {
#pragma unroll
            for (int t = 0; t < NT; ++t) fnx[t] = fl[b + NT * Nx + (long)t * Nx];
        }
        shifted_solve<NT, SCHUR>(tm, sh, g, z);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            up[t] = omega * z[t];
            uout[b + (long)t * Nx] = up[t];
        }
        // residual of u' = omega A^{-1} f: f - A u' + e_1 u'_prev = (1 - omega) f + e_1 u'_prev
#pragma unroll
        for (int t = 0; t < NT; ++t) g2[t] = (1.0 - omega) * g[t];
        g2[0] += prev;
        if (h == 0) {
#pragma unroll
            for (int c = 0; c < NT; ++c) acc[c] = 0.0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int c = 0; c < NT; ++c) acc[c] += tr.P[(h * NT + t) * kNt + c] * g2[t];
        if (h == 1) {
            const long mc = (s0 + k) / 2;
#pragma unroll
            for (int c = 0; c < NT; ++c) fc[mc * NT * Nx + m + (long)c * Nx] = acc[c];
        }
        prev = up[NT - 1];
    }
}

#define STH_NT_SWITCH(KER, GRID, ...)                                                      \
    switch (Nt) {                                                                           \
        case 2: hipLaunchKernelGGL(KER<2>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        case 3: hipLaunchKernelGGL(KER<3>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        case 4: hipLaunchKernelGGL(KER<4>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        case 5: hipLaunchKernelGGL(KER<5>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        case 6: hipLaunchKernelGGL(KER<6>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        case 7: hipLaunchKernelGGL(KER<7>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        case 8: hipLaunchKernelGGL(KER<8>, GRID, dim3(256), 0, st, __VA_ARGS__); break;     \
        default: return hipErrorInvalidValue;                                               \
    }

template <int NT>
static void eig_smooth_launch(dim3 grid, hipStream_t st, int dim, const TimeMix& tm, const double* ktmt,
                              const double* mu1, int n, long Nx, const double* fh, const double* uin, double* uout,
                              long total, double omega, bool zero_guess, const double* ec, const Transfer& tr,
                              const int* guard) {
    const int zg = zero_guess ? 1 : 0;
    if (ec && tm.schur)
        hipLaunchKernelGGL((k_eig_smooth<NT, true, true>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n, Nx, fh, uin,
                           uout, total, omega, zg, ec, tr, guard);
    else if (ec)
        hipLaunchKernelGGL((k_eig_smooth<NT, true, false>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n, Nx, fh,
                           uin, uout, total, omega, zg, ec, tr, guard);
    else if (tm.schur)
        hipLaunchKernelGGL((k_eig_smooth<NT, false, true>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n, Nx, fh,
                           uin, uout, total, omega, zg, ec, tr, guard);
    else
        hipLaunchKernelGGL((k_eig_smooth<NT, false, false>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n, Nx, fh,
                           uin, uout, total, omega, zg, ec, tr, guard);
}

hipError_t launch_eig_smooth(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                             const double* fh, const double* uin, double* uout, long S, double omega,
                             bool zero_guess, const double* ec, const Transfer& tr, hipStream_t st,
                             const int* guard) {
    long Nx = eig_modes(dim, n), total = S * Nx;
    if (total <= 0) return hipSuccess;
    if (ec && zero_guess) return hipErrorInvalidValue;
    dim3 grid((unsigned)((total + 255) / 256));
    switch (Nt) {
#define STH_ES_CASE(NTV) \
        case NTV: eig_smooth_launch<NTV>(grid, st, dim, tm, ktmt, mu1, n, Nx, fh, uin, uout, total, omega, zero_guess, ec, tr, guard); break;
        STH_ES_CASE(2) STH_ES_CASE(3) STH_ES_CASE(4) STH_ES_CASE(5) STH_ES_CASE(6) STH_ES_CASE(7) STH_ES_CASE(8)
#undef STH_ES_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_eig_residual(int dim, int Nt, const double* ktmt, const double* mu1, int n, const double* fh,
                               const double* uh, double* rh, long S, hipStream_t st) {
    long Nx = eig_modes(dim, n), total = S * Nx;
    if (total <= 0) return hipSuccess;
    dim3 grid((unsigned)((total + 255) / 256));
    STH_NT_SWITCH(k_eig_residual, grid, ktmt, dim, mu1, n, Nx, fh, uh, rh, total)
    return hipGetLastError();
}

hipError_t launch_eig_resid_restrict(int dim, int Nt, const Transfer& tr, const double* ktmt, const double* mu1,
                                     int n, const double* fh, const double* uh, double* fc, long Sc,
                                     hipStream_t st) {
    long Nx = eig_modes(dim, n), total = Sc * Nx;
    if (total <= 0) return hipSuccess;
    dim3 grid((unsigned)((total + 255) / 256));
    STH_NT_SWITCH(k_eig_resid_restrict, grid, tr, ktmt, dim, mu1, n, Nx, fh, uh, fc, total)
    return hipGetLastError();
}
#undef STH_NT_SWITCH

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

// ---------------------------------------------------------------------------
// misc
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill(double* v, long len, double val) {
    long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) v[i] = val;
}

hipError_t launch_fill(double* v, long len, double val, hipStream_t st) {
    if (len <= 0) return hipSuccess;
    long blocks = (len + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, v, len, val);
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
    double s = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += 256) s += v[i] * v[i];
    double tot = block_sum_256(s, sh);
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


hipError_t launch_eig_cycle_end(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                                const double* fh, const double* uin, double* uout, double* fc, const Transfer& tr,
                                double omega, long S, int chain, const double* vw, double* partial,
                                long max_partial, double* out, double* out_host, hipStream_t st,
                                const CycleFlag& flag) {
    const long Nx = eig_modes(dim, n);
    if (chain < 2 || chain % 2 || S <= 0 || S % chain || !vw) return hipErrorInvalidValue;
    if (flag.dev && (!flag.host || !flag.thr)) return hipErrorInvalidValue;
    const long total = (S / chain) * Nx;
    const long blocks = (total + 255) / 256;
    if (2 * blocks > max_partial || blocks > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks);
    switch (Nt) {
#define STH_CE_CASE(NTV)                                                                                     \
        case NTV:                                                                                             \
            if (tm.schur)                                                                                     \
                hipLaunchKernelGGL((k_eig_cycle_end<NTV, true>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n, \
                                   Nx, fh, uin, uout, fc, tr, omega, chain, total, vw, partial);              \
            else                                                                                              \
                hipLaunchKernelGGL((k_eig_cycle_end<NTV, false>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1,   \
                                   n, Nx, fh, uin, uout, fc, tr, omega, chain, total, vw, partial);           \
            break;
        STH_CE_CASE(2) STH_CE_CASE(3) STH_CE_CASE(4) STH_CE_CASE(5) STH_CE_CASE(6) STH_CE_CASE(7) STH_CE_CASE(8)
#undef STH_CE_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, (int)blocks, out, out_host, 2, nullptr,
                       flag);
    return hipGetLastError();
}

hipError_t launch_eig_cycle_close(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                                  const double* fh, const double* upre, const double* ec, double* uend,
                                  double* unext, double* fc, const Transfer& tr, double omega, long S, int chain,
                                  const double* vw, double* partial, long max_partial, double* out,
                                  double* out_host, hipStream_t st, const int* guard, const CycleFlag& flag,
                                  bool sums) {
    const long Nx = eig_modes(dim, n);
    if (chain < 2 || chain % 2 || S <= 0 || S % chain || !vw) return hipErrorInvalidValue;
    if (upre == uend || upre == unext || uend == unext) return hipErrorInvalidValue;
    if (flag.dev && (!flag.host || !flag.thr)) return hipErrorInvalidValue;
    const long total = (S / chain) * Nx;
    const long blocks = (total + 255) / 256;
    if (2 * blocks > max_partial || blocks > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks);
    switch (Nt) {
#define STH_CC_CASE(NTV)                                                                                     \
        case NTV:                                                                                             \
            if (tm.schur)                                                                                     \
                hipLaunchKernelGGL((k_eig_cycle_close<NTV, true>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1,  \
                                   n, Nx, fh, upre, ec, uend, unext, fc, tr, omega, chain, total, vw,         \
                                   partial, guard);                                                           \
            else                                                                                              \
                hipLaunchKernelGGL((k_eig_cycle_close<NTV, false>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, \
                                   n, Nx, fh, upre, ec, uend, unext, fc, tr, omega, chain, total, vw,         \
                                   partial, guard);                                                           \
            break;
        STH_CC_CASE(2) STH_CC_CASE(3) STH_CC_CASE(4) STH_CC_CASE(5) STH_CC_CASE(6) STH_CC_CASE(7) STH_CC_CASE(8)
#undef STH_CC_CASE
        default: return hipErrorInvalidValue;
    }
    if (!sums) return hipGetLastError();
    return launch_cycle_sums(dim, n, S, chain, partial, out, out_host, st, guard, flag);
}

hipError_t launch_cycle_sums(int dim, int n, long S, int chain, double* partial, double* out, double* out_host,
                             hipStream_t st, const int* guard, const CycleFlag& flag) {
    const long Nx = eig_modes(dim, n);
    if (chain < 2 || S <= 0 || S % chain) return hipErrorInvalidValue;
    const long blocks = ((S / chain) * Nx + 255) / 256;
    if (flag.dev && (!flag.host || !flag.thr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, (int)blocks, out, out_host, 2, guard,
                       flag);
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


// groups and level-a slabs per thread of the two-level tail pass, or false
// when the shape does not fit it
bool coarse_tail_shape(int Nt, long SA, int* G, int* LA) {
    if (SA < 4 || SA % 4) return false;
    const long g = SA / 2 < 32 ? SA / 2 : 32;
    if (SA % (2 * g)) return false;
    const long la = SA / g;
    if (la > (Nt <= 5 ? 8 : 4)) return false;
    *G = (int)g;
    *LA = (int)la;
    return true;
}

hipError_t launch_eig_coarse_tail(int dim, int Nt, const TimeMix* tma_dev, const TimeMix* tmb_dev, bool schur,
                                  const double* mu1, int n, const double* fa, double* ua,
                                  const Transfer& tr, double omega, long SA, hipStream_t st, const int* guard) {
    const long Nx = eig_modes(dim, n);
    int G = 0, LA = 0;
    if (!coarse_tail_shape(Nt, SA, &G, &LA) || fa == ua) return hipErrorInvalidValue;
    dim3 grid((unsigned)((Nx + 15) / 16)), block((unsigned)(16 * G));
#define STH_CT_GO(NTV, SC, LAMV)                                                                              \
    hipLaunchKernelGGL((k_eig_coarse_tail<NTV, SC, LAMV>), grid, block, 0, st, dim, tma_dev, tmb_dev, mu1, \
                       n, Nx, fa, ua, tr, omega, G, LA, guard)
#define STH_CT_LAM(NTV, SC)                                                                                  \
    if (LA <= 2) STH_CT_GO(NTV, SC, 2);                                                                      \
    else if (LA <= 4) STH_CT_GO(NTV, SC, 4);                                                                 \
    else if (NTV <= 5) STH_CT_GO(NTV, SC, (NTV <= 5 ? 8 : 4));                                               \
    else return hipErrorInvalidValue;
#define STH_CT_CASE(NTV)                                                                                     \
        case NTV:                                                                                             \
            if (schur) { STH_CT_LAM(NTV, true) } else { STH_CT_LAM(NTV, false) }                              \
            break;
    switch (Nt) {
        STH_CT_CASE(2) STH_CT_CASE(3) STH_CT_CASE(4) STH_CT_CASE(5) STH_CT_CASE(6) STH_CT_CASE(7) STH_CT_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef STH_CT_CASE
#undef STH_CT_LAM
#undef STH_CT_GO
    return hipGetLastError();
}

hipError_t launch_eig_down(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                           const double* fl, double* uout, double* fc, const Transfer& tr, double omega, long S,
                           int chain, hipStream_t st, const int* guard) {
    const long Nx = eig_modes(dim, n);
    if (chain < 2 || chain % 2 || S <= 0 || S % chain) return hipErrorInvalidValue;
    const long total = (S / chain) * Nx;
    const long blocks = (total + 255) / 256;
    if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks);
    switch (Nt) {
#define STH_DN_CASE(NTV)                                                                                  \
        case NTV:                                                                                          \
            if (tm.schur)                                                                                  \
                hipLaunchKernelGGL((k_eig_down<NTV, true>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n, Nx, \
                                   fl, uout, fc, tr, omega, chain, total, guard);                          \
            else                                                                                           \
                hipLaunchKernelGGL((k_eig_down<NTV, false>), grid, dim3(256), 0, st, dim, tm, ktmt, mu1, n,    \
                                   Nx, fl, uout, fc, tr, omega, chain, total, guard);                      \
            break;
        STH_DN_CASE(2) STH_DN_CASE(3) STH_DN_CASE(4) STH_DN_CASE(5) STH_DN_CASE(6) STH_DN_CASE(7) STH_DN_CASE(8)
#undef STH_DN_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sth
