// gfx950 kernels of the space-time slab solver: the residual
//   r_n = f_n - A_n u_n + B_n u_{n-1} (eq. equ_linear_system, A_n = K_t (x) M_x
//   + M_t (x) K_x, B_n = N_t (x) M_x with N_t = e_1 e_{N_t}^T, eq. structureAn)
// by sum factorisation: banded 1-D passes of M_1/K_1, then the dense
// N_t x N_t contraction in registers.
#include <atomic>

#include "kernels_common.hpp"

namespace sth {

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
    static std::atomic<bool> attr_set{false};       // set once; the attribute call is idempotent
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t e = hipFuncSetAttribute((const void*)k_residual2d<NT, P, kRY + 2 * P>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_residual2d<NT, P, kRY + P>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set.store(true, std::memory_order_release);
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

// 2-D residual for large images: one wave per (slab, range of columns of x,
// range of YR rows of y), with no LDS and no barrier.  A wave's 64 lanes
// hold 64 consecutive columns; the P lanes at either end only supply the
// neighbours of the others (chunks of 64 - 2P output columns overlap by 2P).
// The wave marches along y: for each input row and time row it applies M_1
// and K_1 along x (neighbours by cross-lane reads), keeps the last 2P+1
// results per time row in registers, and completes each output row with the
// y pass and the temporal contraction.  The next input row is loaded while
// the current one is processed.  With `partial` the block's sum of squares
// of r goes to partial[blockIdx.x] (fixed order).
// waves per SIMD the marching kernel asks for: 4 (at most 128 VGPRs) where
// its windows and time rows are small enough to fit them without spilling
// more than a few registers, else what the compiler picks
template <int NT, int P>
constexpr int march_waves() { return NT <= 4 && (NT + 1) * (2 * P + 1) <= 20 ? 4 : 1; }

template <int NT, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(march_waves<NT, P>())))
void k_residual2d_march(int n, int nxc, int nyr, int YR, long nwaves,
                                                          const double* __restrict__ M1b,
                                                          const double* __restrict__ K1b,
                                                          const double* __restrict__ ktmt,
                                                          const double* __restrict__ f,
                                                          const double* __restrict__ u, double* __restrict__ r,
                                                          long s0, double sign, double* __restrict__ partial) {
    constexpr int B = 2 * P + 1, NR = NT + 1;   // band width; time rows with the coupling row
    constexpr int XS = 64 - 2 * P;              // output columns per wave
    const int lane = threadIdx.x & 63;
    const long w = (long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double ssq = 0.0;
    if (w < nwaves) {
        const long per_slab = (long)nxc * nyr;
        const long s = s0 + w / per_slab;
        const int rem = (int)(w % per_slab);
        const int x = (rem % nxc) * XS - P + lane;
        const bool xin = x >= 0 && x < n;
        const bool xout = xin && lane >= P && lane < 64 - P;
        const int yb = (rem / nxc) * YR, ye = min(n, yb + YR);
        const long Nx = (long)n * n, slab = NT * Nx;
        const bool has_prev = s > 0;
        double bm[B], bk[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            bm[k] = xin ? M1b[(long)x * B + k] : 0.0;
            bk[k] = xin ? K1b[(long)x * B + k] : 0.0;
        }
        // input row y of time row tr (tr = NT: the last time row of slab s - 1)
        double v[NR];
        auto load = [&](int y) {
            const bool yin = y >= 0 && y < n;
#pragma unroll
            for (int tr = 0; tr < NR; ++tr) {
                const bool ok = yin && xin && (tr < NT || has_prev);
                const long base = tr < NT ? s * slab + (long)tr * Nx : (s - 1) * slab + (long)(NT - 1) * Nx;
                v[tr] = ok ? u[base + (long)y * n + x] : 0.0;
            }
        };
        double wa[NR][B], wb[NR][B];
#pragma unroll
        for (int tr = 0; tr < NR; ++tr)
#pragma unroll
            for (int k = 0; k < B; ++k) wa[tr][k] = wb[tr][k] = 0.0;
        // f of output row yo, loaded one input row ahead of its use
        double fv[NT];
        auto load_f = [&](int yo) {
            const bool ok = f && xout && yo >= yb && yo < ye;
            const long off = s * slab + (long)yo * n + x;
#pragma unroll
            for (int t = 0; t < NT; ++t) fv[t] = ok ? f[off + (long)t * Nx] : 0.0;
        };
        load(yb - P);
        load_f(yb - 2 * P);
#pragma unroll 1
        for (int y = yb - P; y < ye + P; ++y) {
            double cv[NR], fc[NT];
#pragma unroll
            for (int tr = 0; tr < NR; ++tr) cv[tr] = v[tr];
#pragma unroll
            for (int t = 0; t < NT; ++t) fc[t] = fv[t];
            if (y + 1 < ye + P) {
                load(y + 1);
                load_f(y + 1 - P);
            }
            // x pass of input row y for every time row, into the windows
            // (lanes whose neighbours fall outside the wave are not output)
#pragma unroll
            for (int tr = 0; tr < NR; ++tr) {
                double a = bm[P] * cv[tr], b = bk[P] * cv[tr];
#pragma unroll
                for (int d = 1; d <= P; ++d) {
                    const double up = __shfl_down(cv[tr], d);    // column x + d
                    const double dn = __shfl_up(cv[tr], d);      // column x - d
                    a += bm[P + d] * up + bm[P - d] * dn;
                    b += bk[P + d] * up + bk[P - d] * dn;
                }
#pragma unroll
                for (int k = 0; k + 1 < B; ++k) {
                    wa[tr][k] = wa[tr][k + 1];
                    wb[tr][k] = wb[tr][k + 1];
                }
                wa[tr][B - 1] = a;
                wb[tr][B - 1] = b;
            }
            // output row y - P: y pass and temporal contraction
            const int yo = y - P;
            if (yo >= yb) {
                double cm[B], ck[B];
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    cm[k] = M1b[(long)yo * B + k];
                    ck[k] = K1b[(long)yo * B + k];
                }
                double acc[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = 0.0;
#pragma unroll
                for (int tr = 0; tr < NT; ++tr) {
                    double Mu = 0.0, Ku = 0.0;
#pragma unroll
                    for (int k = 0; k < B; ++k) {
                        Mu += cm[k] * wa[tr][k];
                        Ku += ck[k] * wa[tr][k] + cm[k] * wb[tr][k];
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[t] -= ktmt[t * kNt + tr] * Mu + ktmt[kNt * kNt + t * kNt + tr] * Ku;
                }
                double Mc = 0.0;                         // B_n u_{n-1}: M_x on the coupling row
#pragma unroll
                for (int k = 0; k < B; ++k) Mc += cm[k] * wa[NT][k];
                acc[0] += Mc;
                if (xout) {
                    const long off = s * slab + (long)yo * n + x;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const double val = fc[t] + sign * acc[t];
                        r[off + (long)t * Nx] = val;
                        ssq += val * val;
                    }
                }
            }
        }
    }
    if (partial) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ssq += __shfl_xor(ssq, off);
        __shared__ double red[4];
        if (lane == 0) red[threadIdx.x >> 6] = ssq;
        __syncthreads();
        if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// rows of y per wave of the marching kernel: the longest range that still
// gives at least 8192 waves (halo rows: 2P per range)
static int march_rows(int n, int p, long ns) {
    const long nxc = (n + 63 - 2 * p) / (64 - 2 * p);
    for (int yr : {128, 64, 32})
        if (ns * nxc * ((n + yr - 1) / yr) >= 8192) return yr;
    return 16;
}

template <int NT, int P>
static hipError_t residual2d_march_launch(int n, const double* M1b, const double* K1b, const double* ktmt,
                                          const double* f, const double* u, double* r, long s0, long ns, double sign,
                                          double* partial, long* nblocks, hipStream_t st) {
    const int nxc = (n + 63 - 2 * P) / (64 - 2 * P), YR = march_rows(n, P, ns), nyr = (n + YR - 1) / YR;
    const long nwaves = ns * nxc * nyr, blocks = (nwaves + 3) / 4;
    if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
    if (nblocks) *nblocks = blocks;
    hipLaunchKernelGGL((k_residual2d_march<NT, P>), dim3((unsigned)blocks), dim3(256), 0, st, n, nxc, nyr, YR, nwaves,
                       M1b, K1b, ktmt, f, u, r, s0, sign, partial);
    return hipGetLastError();
}

template <int P>
static hipError_t residual2d_march_nt(int Nt, int n, const double* M1b, const double* K1b, const double* ktmt,
                                      const double* f, const double* u, double* r, long s0, long ns, double sign,
                                      double* partial, long* nblocks, hipStream_t st) {
#define STH_RM_CASE(NTV)                                                                                    \
    case NTV:                                                                                                \
        if constexpr (2 * (NTV + 1) * (2 * P + 1) <= 64)                                                     \
            return residual2d_march_launch<NTV, P>(n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, partial, nblocks, st); \
        return hipErrorInvalidValue;
    switch (Nt) {
        STH_RM_CASE(2) STH_RM_CASE(3) STH_RM_CASE(4) STH_RM_CASE(5) STH_RM_CASE(6) STH_RM_CASE(7) STH_RM_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef STH_RM_CASE
}

// the marching kernel serves 2-D images of 128 or more columns where its
// windows (2 (N_t + 1)(2p + 1) doubles per lane) fit the registers
static bool residual_marches(int dim, int n, int p, int Nt) {
    return dim == 2 && n >= 128 && p >= 1 && p <= kMaxP && 2 * (Nt + 1) * (2 * p + 1) <= 64;
}

hipError_t launch_residual_norm(int dim, int Nt, int p, int n, const double* M1b, const double* K1b,
                                const double* ktmt, const double* f, const double* u, double* r, long ns,
                                double* partial, long max_partial, double* out, double* out_host, hipStream_t st) {
    if (ns <= 0) return hipSuccess;
    if (!residual_marches(dim, n, p, Nt)) return hipErrorInvalidValue;
    const int nxc = (n + 63 - 2 * p) / (64 - 2 * p), YR = march_rows(n, p, ns), nyr = (n + YR - 1) / YR;
    if ((ns * nxc * nyr + 3) / 4 > max_partial) return hipErrorInvalidValue;
    long blocks = 0;
    hipError_t e;
    switch (p) {
        case 1: e = residual2d_march_nt<1>(Nt, n, M1b, K1b, ktmt, f, u, r, 0, ns, 1.0, partial, &blocks, st); break;
        case 2: e = residual2d_march_nt<2>(Nt, n, M1b, K1b, ktmt, f, u, r, 0, ns, 1.0, partial, &blocks, st); break;
        case 3: e = residual2d_march_nt<3>(Nt, n, M1b, K1b, ktmt, f, u, r, 0, ns, 1.0, partial, &blocks, st); break;
        default: e = residual2d_march_nt<4>(Nt, n, M1b, K1b, ktmt, f, u, r, 0, ns, 1.0, partial, &blocks, st); break;
    }
    if (e != hipSuccess) return e;
    return launch_sum_partials(partial, (int)blocks, out, out_host, 1, nullptr, CycleFlag{}, st);
}

bool residual_norm_fused(int dim, int n, int p, int Nt) { return residual_marches(dim, n, p, Nt); }

hipError_t launch_residual(int dim, int Nt, int p, int n, const double* M1b, const double* K1b,
                           const TimeOp& op, const double* ktmt, const double* f, const double* u, double* r,
                           long s0, long ns, double sign, hipStream_t st) {
    if (ns <= 0) return hipSuccess;
    if (p < 1 || p > kMaxP) return hipErrorInvalidValue;
    if (residual_marches(dim, n, p, Nt)) {
        switch (p) {
            case 1: return residual2d_march_nt<1>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, nullptr, nullptr, st);
            case 2: return residual2d_march_nt<2>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, nullptr, nullptr, st);
            case 3: return residual2d_march_nt<3>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, nullptr, nullptr, st);
            case 4: return residual2d_march_nt<4>(Nt, n, M1b, K1b, ktmt, f, u, r, s0, ns, sign, nullptr, nullptr, st);
        }
    }
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

}  // namespace sth
