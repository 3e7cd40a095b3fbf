// gfx950 kernels of the space-time slab solver: the spatial eigenbasis
// transforms of 2-D images with the whole image in LDS (eq.
// equ:ST:generalDecompA with fast diagonalisation of K_x + lambda M_x), in
// FP64, FP32 and BF16x3 MFMA, and the exact B-spline residual norm of an
// eigenbasis vector through the Gram matrix G = C^T C.
#include <atomic>
#include <type_traits>

#include "kernels_common.hpp"

namespace sth {

// ---------------------------------------------------------------------------
// Both spatial axes of a 2-D image in one kernel: U (padded to NP x NP) and
// one image stay in LDS; every block walks over images.  DIR 0 (forward):
// out = U^T R U.  DIR 1 (inverse): Z = U Y U^T, then the epilogue EPI
// (0 store, 1 out += alpha Z, 2 out = alpha Z).  Eight waves share the
// NT16 x NT16 output tiles of each GEMM; the intermediate product goes back
// into the image buffer.  CT is the compute type: double (MFMA f64 16x16x4)
// or float (MFMA f32 16x16x4, FP32 accumulation); global data stay FP64.
// ---------------------------------------------------------------------------
template <typename CT, int DIR, int NT16, int EPI, bool CORE, typename TI, typename TO>
__global__ __launch_bounds__(512) void k_xform2d(const TI* __restrict__ in, TO* __restrict__ out,
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
        const TI* src = in + img * ldi;
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
                TO* dst = out + img * ldo;
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
        TO* dst = out + img * ldo;
        auto put = [&](int i, int j, double v) {
            TO* o = dst + (long)i * n + j;
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
template <typename CT, int DIR, int NT16, int EPI, bool CORE, typename TI, typename TO>
static hipError_t xform2d_go(const TI* in, TO* out, const double* Upad, int n, long nimg, double alpha,
                             hipStream_t st, long* nblocks, const int* guard, long ldi, long ldo) {
    size_t shm = sizeof(CT) * 2 * (size_t)TileLds<CT, NT16>::SIZE;
    static std::atomic<bool> attr_set{false};       // set once; the attribute call is idempotent
    if (!attr_set.load(std::memory_order_acquire)) {
        // exactly the dynamic size: the block-wide vote holds a little static LDS
        hipError_t e = hipFuncSetAttribute((const void*)k_xform2d<CT, DIR, NT16, EPI, CORE, TI, TO>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_set.store(true, std::memory_order_release);
    }
    long blocks = persistent_blocks(shm, nimg);
    if (nblocks) *nblocks = blocks;
    hipLaunchKernelGGL((k_xform2d<CT, DIR, NT16, EPI, CORE, TI, TO>), dim3((unsigned)blocks), dim3(512), shm, st, in, out,
                       Upad, n, nimg, alpha, guard, ldi, ldo);
    return hipGetLastError();
}

template <typename CT, int DIR, int NT16, int EPI, typename TI, typename TO>
static hipError_t xform2d_launch(const TI* in, TO* out, const double* Upad, int n, long nimg, double alpha,
                                 hipStream_t st, long* nblocks = nullptr, const int* guard = nullptr,
                                 long ldi = 0, long ldo = 0) {
    if (n > 16 * NT16 || n <= 16 * (NT16 - 1)) return hipErrorInvalidValue;
    if (ldi == 0) ldi = (long)n * n;
    if (ldo == 0) ldo = (long)n * n;
    if (ldi < (long)n * n || ldo < (long)n * n) return hipErrorInvalidValue;
    if constexpr (kXform2dEdge<NT16>) {
        if (xform2d_core_tiles<NT16>(n) < NT16)
            return xform2d_go<CT, DIR, NT16, EPI, true, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
    }
    return xform2d_go<CT, DIR, NT16, EPI, false, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
}

template <typename CT, int DIR, int EPI, typename TI = double, typename TO = double>
static hipError_t xform2d_np(const TI* in, TO* out, const double* Upad, int n, int np, long nimg,
                             double alpha, hipStream_t st, long* nblocks = nullptr, const int* guard = nullptr,
                             long ldi = 0, long ldo = 0) {
    switch (np / 16) {
        case 1: return xform2d_launch<CT, DIR, 1, EPI, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 2: return xform2d_launch<CT, DIR, 2, EPI, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 3: return xform2d_launch<CT, DIR, 3, EPI, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 4: return xform2d_launch<CT, DIR, 4, EPI, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 5: return xform2d_launch<CT, DIR, 5, EPI, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        case 6: return xform2d_launch<CT, DIR, 6, EPI, TI, TO>(in, out, Upad, n, nimg, alpha, st, nblocks, guard, ldi, ldo);
        default: return hipErrorInvalidValue;
    }
}

template <typename CT>
static hipError_t xform2d_prec(int dir, int epi, const double* in, double* out, const double* Upad, int n, int np,
                               long nimg, double alpha, hipStream_t st, const int* guard, long ldi, long ldo,
                               int io_f32) {
    if (io_f32) {
        // FP32 eigenbasis vectors (FP32 transforms only): the forward
        // transform writes them, the inverse reads them
        if (!std::is_same<CT, float>::value) return hipErrorInvalidValue;
        if (dir == 0 && io_f32 == 2)
            return xform2d_np<CT, 0, 0, double, float>(in, (float*)out, Upad, n, np, nimg, 1.0, st, nullptr, guard,
                                                       ldi, ldo);
        if (dir == 1 && io_f32 == 1 && epi == 0)
            return xform2d_np<CT, 1, 0, float, double>((const float*)in, out, Upad, n, np, nimg, alpha, st, nullptr,
                                                       guard, ldi, ldo);
        if (dir == 1 && io_f32 == 1 && epi == 1)
            return xform2d_np<CT, 1, 1, float, double>((const float*)in, out, Upad, n, np, nimg, alpha, st, nullptr,
                                                       guard, ldi, ldo);
        return hipErrorInvalidValue;
    }
    if (dir == 0) return xform2d_np<CT, 0, 0>(in, out, Upad, n, np, nimg, 1.0, st, nullptr, guard, ldi, ldo);
    if (epi == 0) return xform2d_np<CT, 1, 0>(in, out, Upad, n, np, nimg, alpha, st, nullptr, guard, ldi, ldo);
    if (epi == 1) return xform2d_np<CT, 1, 1>(in, out, Upad, n, np, nimg, alpha, st, nullptr, guard, ldi, ldo);
    if (epi == 2) return xform2d_np<CT, 1, 2>(in, out, Upad, n, np, nimg, alpha, st, nullptr, guard, ldi, ldo);
    return hipErrorInvalidValue;
}
template <int NT16, int EPI, typename TI, typename TO>
__global__ __launch_bounds__(512) void k_xform2d_bf16x3(const TI* __restrict__ in, TO* __restrict__ out,
                                                        const double* __restrict__ Mpad, int n, long nimg,
                                                        double alpha, const int* guard, long ldi, long ldo) {
    if (guard_off(guard)) return;
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
        const TI* src = in + img * ldi;
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
            const int i = tid + 512 * k, r = i / NP, c = i % NP;
            if (i < NP * NP) split_bf16(pre[k], &Ih[r * LDB + c], &Il[r * LDB + c]);
            nz |= pre[k] != 0.0;
        }
        if (img + gridDim.x < nimg) load_img(img + gridDim.x);
        // an image of zeros maps to zeros
        if (!__syncthreads_or(nz)) {
            if (EPI != 1) {
                TO* dst = out + img * ldo;
                for (long i = tid; i < nn; i += 512) dst[i] = 0.0;
            }
            continue;
        }
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
        TO* dst = out + img * ldo;
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
                        TO* o = dst + (long)i * n + j;
                        if (EPI == 0) *o = v;
                        else if (EPI == 1) *o += alpha * v;
                        else *o = alpha * v;
                    }
                }
            }
        }
    }
}

template <int NT16, int EPI, typename TI, typename TO>
static hipError_t xform2d_bf16_launch(const TI* in, TO* out, const double* Mpad, int n, long nimg,
                                      double alpha, hipStream_t st, const int* guard, long ldi, long ldo) {
    constexpr int NP = NT16 * 16;
    size_t shm = sizeof(unsigned short) * 4 * (size_t)NP * (NP + 8);
    static std::atomic<bool> attr_set{false};       // set once; the attribute call is idempotent
    if (!attr_set.load(std::memory_order_acquire)) {
        // exactly the dynamic size: the block-wide vote holds a little static LDS
        hipError_t e = hipFuncSetAttribute((const void*)k_xform2d_bf16x3<NT16, EPI, TI, TO>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_set.store(true, std::memory_order_release);
    }
    long blocks = persistent_blocks(shm, nimg);
    hipLaunchKernelGGL((k_xform2d_bf16x3<NT16, EPI, TI, TO>), dim3((unsigned)blocks), dim3(512), shm, st, in, out, Mpad,
                       n, nimg, alpha, guard, ldi, ldo);
    return hipGetLastError();
}

template <int EPI, typename TI = double, typename TO = double>
static hipError_t xform2d_bf16_np(const TI* in, TO* out, const double* Mpad, int n, int np, long nimg,
                                  double alpha, hipStream_t st, const int* guard, long ldi, long ldo) {
    switch (np / 16) {
        case 1: return xform2d_bf16_launch<1, EPI, TI, TO>(in, out, Mpad, n, nimg, alpha, st, guard, ldi, ldo);
        case 2: return xform2d_bf16_launch<2, EPI, TI, TO>(in, out, Mpad, n, nimg, alpha, st, guard, ldi, ldo);
        case 3: return xform2d_bf16_launch<3, EPI, TI, TO>(in, out, Mpad, n, nimg, alpha, st, guard, ldi, ldo);
        case 4: return xform2d_bf16_launch<4, EPI, TI, TO>(in, out, Mpad, n, nimg, alpha, st, guard, ldi, ldo);
        case 5: return xform2d_bf16_launch<5, EPI, TI, TO>(in, out, Mpad, n, nimg, alpha, st, guard, ldi, ldo);
        case 6: return xform2d_bf16_launch<6, EPI, TI, TO>(in, out, Mpad, n, nimg, alpha, st, guard, ldi, ldo);
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
template <int NT16, bool CORE>
static hipError_t gram_norm2d_go(const double* in, const double* Gpad, int n, long nimg, double* partial,
                                 int max_blocks, double* out, double* out_host, hipStream_t st,
                                 const CycleFlag& flag, long ldi) {
    const size_t shm = sizeof(double) * 2 * (size_t)TileLds<double, NT16>::SIZE;
    static std::atomic<bool> attr_set{false};       // set once; the attribute call is idempotent
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t e = hipFuncSetAttribute((const void*)k_gram_norm2d<NT16, CORE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr_set.store(true, std::memory_order_release);
    }
    const long blocks = persistent_blocks(shm, nimg);
    if (blocks > max_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gram_norm2d<NT16, CORE>), dim3((unsigned)blocks), dim3(512), shm, st, in, Gpad, n, nimg,
                       partial, ldi);
    return launch_sum_partials(partial, (int)blocks, out, out_host, 1, nullptr, flag, st);
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
                          int np, long nimg, double alpha, hipStream_t st, const int* guard, long ldi, long ldo,
                          int io_f32) {
    if (nimg <= 0) return hipSuccess;
    if (!xform2d_supported(np)) return hipErrorInvalidValue;
    if (prec == 0)
        return xform2d_prec<double>(dir, epi, in, out, Upad, n, np, nimg, alpha, st, guard, ldi, ldo, io_f32);
    if (prec == 1)
        return xform2d_prec<float>(dir, epi, in, out, Upad, n, np, nimg, alpha, st, guard, ldi, ldo, io_f32);
    return hipErrorInvalidValue;
}

hipError_t launch_xform2d_bf16x3(int epi, const double* in, double* out, const double* Mpad, int n, int np,
                                 long nimg, double alpha, hipStream_t st, const int* guard, long ldi, long ldo,
                                 int io_f32) {
    if (nimg <= 0) return hipSuccess;
    if (!xform2d_supported(np) || n > np || n <= np - 16) return hipErrorInvalidValue;
    if (ldi == 0) ldi = (long)n * n;
    if (ldo == 0) ldo = (long)n * n;
    if (ldi < (long)n * n || ldo < (long)n * n) return hipErrorInvalidValue;
    if (io_f32 == 2 && epi == 0)             // forward transform into FP32 eigenbasis vectors
        return xform2d_bf16_np<0, double, float>(in, (float*)out, Mpad, n, np, nimg, 1.0, st, guard, ldi, ldo);
    if (io_f32 == 1 && epi == 0)             // inverse transform from FP32 eigenbasis vectors
        return xform2d_bf16_np<0, float, double>((const float*)in, out, Mpad, n, np, nimg, 1.0, st, guard, ldi, ldo);
    if (io_f32 == 1 && epi == 1)
        return xform2d_bf16_np<1, float, double>((const float*)in, out, Mpad, n, np, nimg, alpha, st, guard, ldi,
                                                 ldo);
    if (io_f32) return hipErrorInvalidValue;
    if (epi == 0) return xform2d_bf16_np<0>(in, out, Mpad, n, np, nimg, 1.0, st, guard, ldi, ldo);
    if (epi == 1) return xform2d_bf16_np<1>(in, out, Mpad, n, np, nimg, alpha, st, guard, ldi, ldo);
    if (epi == 2) return xform2d_bf16_np<2>(in, out, Mpad, n, np, nimg, alpha, st, guard, ldi, ldo);
    return hipErrorInvalidValue;
}

}  // namespace sth
