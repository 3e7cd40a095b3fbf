// gfx950 kernels of the space-time slab solver: the spatial eigenbasis
// transforms one axis at a time (3-D, and 2-D images too large for the
// LDS-resident kernels) as MFMA GEMMs in FP64, FP32 and BF16x3.  The
// launchers take the panel kernels (transform matrix in LDS) for np <= 256;
// the kernels here serve larger n.
#include "kernels_common.hpp"

namespace sth {

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
                                                 double alpha, const int* guard) {
    if (guard_off(guard)) return;
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
        int nz = 0;
        for (int i = threadIdx.x; i < 64 * 16; i += 256) {
            int l = i >> 4, kk = i & 15;
            long line = line0 + l;
            int k = k0 + kk;
            const double v = (line < lines && k < n) ? in[line * n + k] : 0.0;
            nz |= v != 0.0;
            in_s[ia(l, kk)] = (CT)v;
        }
        for (int i = threadIdx.x; i < 16 * 128; i += 256) {
            int kk = i >> 7, jj = i & 127;
            int j = j0 + jj;
            T_s[ta(kk, jj)] = (CT)((j < np) ? T[(long)(k0 + kk) * np + j] : 0.0);
        }
        // a k-chunk of zeros (e.g. a zero initial guess) adds nothing: the
        // block-wide vote skips its MFMAs
        if (__syncthreads_or(nz)) {
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) {
                CT a = in_s[ia(wave * 16 + lr, kq * 4 + lk)];
#pragma unroll
                for (int jt = 0; jt < 8; ++jt) {
                    if (jt < njt) acc[jt] = M::op(a, T_s[ta(kq * 4 + lk, jt * 16 + lr)], acc[jt]);
                }
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
                                                 int nib, int njb, const int* guard) {
    if (guard_off(guard)) return;
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
        int nz = 0;
        for (int i = threadIdx.x; i < 16 * 64; i += 256) {
            int kk = i >> 6, ii = i & 63;
            int k = k0 + kk;
            long ig = i0 + ii;
            const double v = (k < n && ig < inner) ? inb[(long)k * inner + ig] : 0.0;
            nz |= v != 0.0;
            in_s[sa(kk, ii)] = (CT)v;
            int j = j0 + ii;
            T_s[sa(kk, ii)] = (CT)((j < np) ? T[(long)k * np + j] : 0.0);
        }
        // k-chunks of zeros are skipped (block-wide vote)
        if (__syncthreads_or(nz) && active) {
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
                                                        double alpha, const int* guard) {
    if (guard_off(guard)) return;
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
        int nz = 0;
        for (int i = threadIdx.x; i < 64 * 16; i += 256) {
            int l = i >> 4, kk = i & 15;
            long line = line0 + l;
            int k = k0 + kk;
            const double v = (line < lines && k < n) ? in[line * n + k] : 0.0;
            nz |= v != 0.0;
            split_bf16(v, &ih[l][kk], &il[l][kk]);
        }
        for (int i = threadIdx.x; i < 16 * 128; i += 256) {
            int kk = i >> 7, jj = i & 127;
            int j = j0 + jj;
            split_bf16((j < np) ? T[(long)(k0 + kk) * np + j] : 0.0, &th[jj][kk], &tl[jj][kk]);
        }
        if (!__syncthreads_or(nz)) {          // a k-chunk of zeros adds nothing
            __syncthreads();
            continue;
        }
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
                                                        int nib, int njb, const int* guard) {
    if (guard_off(guard)) return;
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
        int nz = 0;
        for (int i = threadIdx.x; i < 16 * 64; i += 256) {
            int kk = i >> 6, ii = i & 63;
            int k = k0 + kk;
            long ig = i0 + ii;
            const double v = (k < n && ig < inner) ? inb[(long)k * inner + ig] : 0.0;
            nz |= v != 0.0;
            split_bf16(v, &ih[ii][kk], &il[ii][kk]);
            int j = j0 + ii;
            split_bf16((j < np) ? T[(long)k * np + j] : 0.0, &th[ii][kk], &tl[ii][kk]);
        }
        if (__syncthreads_or(nz) && active) {          // k-chunks of zeros are skipped
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
                       int np, long lines, double alpha, const int* guard) {
    if (epi == 0)
        hipLaunchKernelGGL((k_xform_x<CT, 0>), grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha, guard);
    else if (epi == 1)
        hipLaunchKernelGGL((k_xform_x<CT, 1>), grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha, guard);
    else
        hipLaunchKernelGGL((k_xform_x<CT, 2>), grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha, guard);
}

bool xform_split_supported(int n) { return xform_panel_split_supported(n); }

hipError_t launch_xform_x(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                          long lines, double alpha, hipStream_t st, const int* guard, int sym, int io) {
    if (lines <= 0) return hipSuccess;
    if (epi < 0 || epi > 2 || prec < 0 || prec > 2) return hipErrorInvalidValue;
    if (xform_panel_supported(np))
        return launch_xform_panel_x_io(prec, epi, in, out, T, n, np, lines, alpha, st, guard, sym, io);
    if (sym || io) return hipErrorInvalidValue;
    dim3 grid((unsigned)((lines + 63) / 64), (unsigned)((np + 127) / 128));
    if (prec == 0) xform_x_ct<double>(epi, grid, st, in, out, T, n, np, lines, alpha, guard);
    else if (prec == 1) xform_x_ct<float>(epi, grid, st, in, out, T, n, np, lines, alpha, guard);
    else if (epi == 0)
        hipLaunchKernelGGL(k_xform_x_bf16x3<0>, grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha, guard);
    else if (epi == 1)
        hipLaunchKernelGGL(k_xform_x_bf16x3<1>, grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha, guard);
    else
        hipLaunchKernelGGL(k_xform_x_bf16x3<2>, grid, dim3(256), 0, st, in, out, T, n, np, lines, alpha, guard);
    return hipGetLastError();
}

hipError_t launch_xform_s(int prec, const double* in, double* out, const double* T, int n, int np,
                          long nbatch, long inner, hipStream_t st, const int* guard, int io_f32, int sym) {
    if (nbatch <= 0) return hipSuccess;
    if (prec < 0 || prec > 2) return hipErrorInvalidValue;
    if (xform_panel_supported(np))
        return launch_xform_panel_s(prec, in, out, T, n, np, nbatch, inner, st, guard, io_f32, sym);
    if (sym) return hipErrorInvalidValue;
    if (io_f32) return hipErrorInvalidValue;      // FP32 storage: the panel kernels only
    int nib = (int)((inner + 63) / 64), njb = (np + 63) / 64;
    long blocks = nbatch * nib * njb;
    if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
    if (prec == 0)
        hipLaunchKernelGGL(k_xform_s<double>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, n, np, inner,
                           nib, njb, guard);
    else if (prec == 1)
        hipLaunchKernelGGL(k_xform_s<float>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, n, np, inner,
                           nib, njb, guard);
    else
        hipLaunchKernelGGL(k_xform_s_bf16x3, dim3((unsigned)blocks), dim3(256), 0, st, in, out, T, n, np, inner,
                           nib, njb, guard);
    return hipGetLastError();
}

}  // namespace sth
