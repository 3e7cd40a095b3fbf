// gfx950 kernels of the space-time slab solver: the spatial eigenbasis
// transforms one axis at a time (eq. equ:ST:generalDecompA with fast
// diagonalisation of K_x + lambda M_x) for np <= 256 (a multiple of 32), as
// MFMA GEMMs with the
// transform matrix held in LDS and the data streamed through registers.
//
// A block stages one panel of PW output columns of the (padded) transform
// matrix T, all of its rows, in LDS once; then each wave works on its own
// 16-row tiles of the data with no further barrier.  A tile's data (16 rows
// x np) goes through registers in groups of 64 k (four consecutive k per
// lane and chunk of 16); the loads of the next group are in flight while the
// current one is in the MFMAs.  Inside a chunk of 16, MFMA step s of lane
// group g (lanes 16g..16g+15) takes k = 16c + 4g + s: every lane supplies
// four consecutive k of its row, and the panel rows are read in the same
// order, which leaves the sum over k unchanged.
//
//  x axis (contiguous): out[line][j] (EPI) sum_k in[line][k] T[k][j];
//    MFMA A = data (rows = lines), B = panel (columns = j).
//  strided axis: out[b][j][i] = sum_k T[k][j] in[b][k][i];
//    MFMA A = panel^T (rows = j), B = data (columns = i), so that the
//    results of a lane group are 16 consecutive i (coalesced stores).
//
// Blocks are persistent.  With P panels (np / PW), the P blocks that handle
// the same data tiles have block ids b, b + 8, b + 16, ... so that they sit
// on the same XCD (block ids go round-robin over the eight XCDs) and share
// the data in its L2.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "kernels_common.hpp"

namespace sth {

constexpr int kPanelThreads = 512;              // eight waves
constexpr int kPanelWaves = kPanelThreads / 64;

// compute types of the panel kernels
struct PanelF64 {};
struct PanelF32 {};
struct PanelBf16x3 {};

template <typename C> struct PanelTraits;
template <> struct PanelTraits<PanelF64> { static constexpr int PW = 64; };
template <> struct PanelTraits<PanelF32> { static constexpr int PW = 128; };
template <> struct PanelTraits<PanelBf16x3> { static constexpr int PW = 128; };

// LDS bytes of a panel of pw columns and kp rows
template <typename C> static size_t panel_lds(int kp, int pw) {
    if constexpr (std::is_same<C, PanelF64>::value) return sizeof(double) * (size_t)kp * pw;
    else if constexpr (std::is_same<C, PanelF32>::value) return sizeof(float) * (size_t)kp * pw;
    else return 2 * sizeof(unsigned short) * (size_t)pw * (kp + 4);
}

template <typename C, int PW, bool XAXIS, int EPI, typename TI, typename TO, int SYM>
__global__ __launch_bounds__(kPanelThreads) void k_xform_panel(const TI* __restrict__ in, TO* __restrict__ out,
                                                               const double* __restrict__ T, int n, int np,
                                                               int npanel, long nrows, long inner, long ntiles,
                                                               double alpha, const int* guard) {
    if (guard_off(guard)) return;
    constexpr int pw = PW;                       // panel width (output columns)
    constexpr int NJT = PW / 16;                 // column tiles per wave
    constexpr bool F64 = std::is_same<C, PanelF64>::value;
    constexpr bool BF = std::is_same<C, PanelBf16x3>::value;
    const int hn = n / 2;
    // panel rows (k), zero from np on; with the even/odd split (np = n,
    // n / 2 a multiple of 64) the forward transform sums over k < n / 2
    const int KP = SYM == 1 ? hn : (SYM == 2 ? n : 64 * ((np + 63) / 64));
    const int ngroups = KP / 64;                 // groups of four chunks of 16 k
    extern __shared__ double sm_raw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: tile bookkeeping in scalars
    const int lr = lane & 15, lg = lane >> 4;
    // persistent block -> (panel, tile stream); see the file comment
    const int b = blockIdx.x, xcd = b & 7, q = b >> 3;
    const int panel = q % npanel;
    const long stream = (long)(q / npanel) * 8 + xcd;
    const long nstream = (long)gridDim.x / npanel;
    const int j0 = panel * pw;
    // stage the panel: T[k][j0 + jj], k < KP (rows from np on are zero)
    if constexpr (BF) {
        unsigned short* th = reinterpret_cast<unsigned short*>(sm_raw);
        unsigned short* tl = th + (size_t)pw * (KP + 4);
        for (int i = tid; i < KP * pw; i += kPanelThreads) {
            const int k = i / pw, jj = i % pw;
            split_bf16(k < np ? T[(long)k * np + j0 + jj] : 0.0, &th[jj * (KP + 4) + k], &tl[jj * (KP + 4) + k]);
        }
    } else {
        using CT = typename std::conditional<F64, double, float>::type;
        CT* tp = reinterpret_cast<CT*>(sm_raw);
        for (int i = tid; i < KP * pw; i += kPanelThreads) {
            const int k = i / pw, jj = i % pw;
            tp[k * pw + jj] = (CT)(k < np ? T[(long)k * np + j0 + jj] : 0.0);
        }
    }
    __syncthreads();
    // forward split: columns [0, n / 2) are even modes, fed x_k + x_{n-1-k};
    // columns [n / 2, n) odd modes, fed x_k - x_{n-1-k}
    const double sgn = (SYM == 1 && j0 >= hn) ? -1.0 : 1.0;
    // tiles: x axis, tile t = lines 16t..16t+15; strided axis, tile t =
    // (batch t / itb, columns 16 (t % itb) .. +15) with itb = ceil(inner / 16)
    const long itb = XAXIS ? 1 : (inner + 15) / 16;
    // a wave's tile: element (row lr, k) at in + rbase + lr * rs + k * ks
    struct Tile {
        long t, rbase, rows_left, bbase, i0;
        bool ok, row_ok;                         // the tile exists; row lr of it does
    };
    const long rs = XAXIS ? n : 1, ks = XAXIS ? 1 : inner;
    auto tile_of = [&](long grp) {
        Tile c;
        c.t = grp * kPanelWaves + wave;
        c.ok = c.t < ntiles;
        c.bbase = 0;
        c.i0 = 0;
        if (XAXIS) {
            c.rbase = c.t * 16 * (long)n;
            c.rows_left = nrows - c.t * 16;
        } else {
            const long bt = c.t / itb;
            c.i0 = (c.t % itb) * 16;
            c.bbase = bt * (long)n * inner;
            c.rbase = c.bbase + c.i0;
            c.rows_left = inner - c.i0;
        }
        c.row_ok = c.ok && lr < c.rows_left;
        return c;
    };
    // lane (lr, lg) holds k = 64 gi + 16 c + 4 lg + e of row lr.  The
    // loads of group gi + 1 go to ra (and, folding, rb: x_{n-1-k}) and
    // are in flight while group gi is in the MFMAs; only then are they
    // converted (and folded) into cur, held in the compute precision
    // (FP32 for the FP32 and BF16x3 kernels).
    using DT = typename std::conditional<F64, double, float>::type;
    TI ra[4][4], rb[SYM == 1 ? 4 : 1][4];
    // addresses: a wave-uniform base (scalar registers) plus a 32-bit lane
    // offset, the same for all sixteen loads of a group
    const unsigned loff = (unsigned)(lr * rs + 4 * lg * ks);
    const unsigned loff_m = (unsigned)(lr * rs + (12 - 4 * lg) * ks);   // mirrored rows, from k + 12
    auto load = [&](const Tile& tl_, int gi) {
        const int kb = 64 * gi + 4 * lg;
        const int kend = SYM == 1 ? hn : n;
        const bool row_ok = tl_.row_ok;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = row_ok && kb + 16 * c + e < kend;
                // element k = 64 gi + 16 c + e + 4 lg of row lr
                const TI* pu = in + tl_.rbase + (long)(64 * gi + 16 * c + e) * ks;
                ra[c][e] = ok ? pu[loff] : (TI)0;
                if constexpr (SYM == 1) {
                    // element n - 1 - k
                    const TI* pm = in + tl_.rbase + (long)(n - 1 - 12 - 64 * gi - 16 * c - e) * ks;
                    rb[c][e] = ok ? pm[loff_m] : (TI)0;
                }
            }
    };
    DT cur[4][4];
    auto settle = [&]() {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if constexpr (SYM == 1) cur[c][e] = (DT)((double)ra[c][e] + sgn * (double)rb[c][e]);
                else cur[c][e] = (DT)ra[c][e];
            }
    };
    // output j0 + jl of tile row il (x axis: line 16 t + il; strided
    // axis: column i0 + il) from v; with the inverse split v + w there and
    // v - w at the mirrored output n - 1 - j
    // The update epilogue (EPI 1) reads the tile's old outputs first, all of
    // them, so that their loads overlap (old[0], and old[1] at the mirror).
    constexpr int NS = SYM == 2 ? 2 : 1;
    auto put = [&](TO* o, double v, double old) {
        if (EPI == 0) *o = v;
        else if (EPI == 1) *o = old + alpha * v;
        else *o = alpha * v;
    };
    auto emit = [&](const Tile& tc, int jl, int il, double v, double w, const double* old) {
        const int j = j0 + jl;
        if (il >= tc.rows_left || j >= n) return;
        TO* o = XAXIS ? out + (tc.t * 16 + il) * (long)n : out + tc.bbase + tc.i0 + il;
        const long js = XAXIS ? 1 : inner;
        if (SYM == 2) {
            put(o + j * js, v + w, old[0]);
            put(o + (n - 1 - j) * js, v - w, old[NS - 1]);
        } else {
            put(o + j * js, v, old[0]);
        }
    };
    auto gather = [&](const Tile& tc, int jl, int il, double* old) {
        const int j = j0 + jl;
        if (il >= tc.rows_left || j >= n) return;
        const TO* o = XAXIS ? out + (tc.t * 16 + il) * (long)n : out + tc.bbase + tc.i0 + il;
        const long js = XAXIS ? 1 : inner;
        old[0] = o[j * js];
        if (SYM == 2) old[NS - 1] = o[(n - 1 - j) * js];
    };
    // the first group of a wave's next tile is loaded during the last group
    // of its current one
    long grp = stream;
    Tile tn = tile_of(grp);
    if (tn.ok) load(tn, 0);
    for (;; grp += nstream) {
        const Tile tc = tn;
        if (!tc.ok) break;
        settle();
        tn = tile_of(grp + nstream);
        if constexpr (BF) {
            const unsigned short* th = reinterpret_cast<const unsigned short*>(sm_raw);
            const unsigned short* tl = th + (size_t)pw * (KP + 4);
            f4 acc[NJT], acc2[SYM == 2 ? NJT : 1];
#pragma unroll
            for (int jt = 0; jt < NJT; ++jt) acc[jt] = f4{0.f, 0.f, 0.f, 0.f};
            if constexpr (SYM == 2) {
#pragma unroll
                for (int jt = 0; jt < NJT; ++jt) acc2[jt] = f4{0.f, 0.f, 0.f, 0.f};
            }
            auto mma = [&](int gi, auto& A) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    s4 dh, dl;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        unsigned short hi, lo;
                        split_bf16(cur[c][e], &hi, &lo);
                        dh[e] = (short)hi;
                        dl[e] = (short)lo;
                    }
#pragma unroll
                    for (int jt = 0; jt < NJT; ++jt) {
                        const int o = (jt * 16 + lr) * (KP + 4) + 64 * gi + 16 * c + 4 * lg;
                        const s4 bh = *reinterpret_cast<const s4*>(&th[o]);
                        const s4 bl = *reinterpret_cast<const s4*>(&tl[o]);
                        if (XAXIS) {
                            A[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dh, bh, A[jt], 0, 0, 0);
                            A[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dh, bl, A[jt], 0, 0, 0);
                            A[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dl, bh, A[jt], 0, 0, 0);
                        } else {
                            A[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bh, dh, A[jt], 0, 0, 0);
                            A[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bl, dh, A[jt], 0, 0, 0);
                            A[jt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bh, dl, A[jt], 0, 0, 0);
                        }
                    }
                    // keep each chunk's operand reads with its MFMAs
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
#pragma unroll 1
            for (int gi = 0; gi < ngroups; ++gi) {
                if (gi + 1 < ngroups) load(tc, gi + 1);
                else if (tn.ok) load(tn, 0);
                int nz = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) nz |= cur[c][e] != (DT)0;
                if (__any(nz)) {                 // a group of zeros adds nothing
                    if constexpr (SYM == 2) {
                        // inverse split: even modes (k < n / 2) into acc, odd into acc2
                        if (gi < ngroups / 2) mma(gi, acc);
                        else mma(gi, acc2);
                    } else {
                        mma(gi, acc);
                    }
                }
                if (gi + 1 < ngroups) settle();
            }
            // D[4 lg + r][lr]: x axis (line, j), strided axis (j, i)
            double old[EPI == 1 ? NJT : 1][4][NS] = {};
            if constexpr (EPI == 1) {
#pragma unroll
                for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        gather(tc, XAXIS ? jt * 16 + lr : jt * 16 + 4 * lg + r, XAXIS ? 4 * lg + r : lr, old[jt][r]);
            }
#pragma unroll
            for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    emit(tc, XAXIS ? jt * 16 + lr : jt * 16 + 4 * lg + r, XAXIS ? 4 * lg + r : lr, (double)acc[jt][r],
                         SYM == 2 ? (double)acc2[SYM == 2 ? jt : 0][r] : 0.0, old[EPI == 1 ? jt : 0][r]);
            (void)acc2;
        } else {
            using CT = typename std::conditional<F64, double, float>::type;
            using M = Mfma16<CT>;
            typedef typename M::acc_t acc_t;
            const CT* tp = reinterpret_cast<const CT*>(sm_raw);
            acc_t acc[NJT], acc2[SYM == 2 ? NJT : 1];
#pragma unroll
            for (int jt = 0; jt < NJT; ++jt) acc[jt] = acc_t{0, 0, 0, 0};
            if constexpr (SYM == 2) {
#pragma unroll
                for (int jt = 0; jt < NJT; ++jt) acc2[jt] = acc_t{0, 0, 0, 0};
            }
            auto mma = [&](int gi, auto& A) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const CT d = (CT)cur[c][s];
                        const CT* row = tp + (64 * gi + 16 * c + 4 * lg + s) * pw + lr;
#pragma unroll
                        for (int jt = 0; jt < NJT; ++jt) {
                            const CT w = row[jt * 16];
                            A[jt] = XAXIS ? M::op(d, w, A[jt]) : M::op(w, d, A[jt]);
                        }
                    }
                    // keep each chunk's operand reads with its MFMAs
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
#pragma unroll 1
            for (int gi = 0; gi < ngroups; ++gi) {
                if (gi + 1 < ngroups) load(tc, gi + 1);
                else if (tn.ok) load(tn, 0);
                int nz = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) nz |= cur[c][e] != (DT)0;
                if (__any(nz)) {                 // a group of zeros adds nothing
                    if constexpr (SYM == 2) {
                        // inverse split: even modes (k < n / 2) into acc, odd into acc2
                        if (gi < ngroups / 2) mma(gi, acc);
                        else mma(gi, acc2);
                    } else {
                        mma(gi, acc);
                    }
                }
                if (gi + 1 < ngroups) settle();
            }
            double old[EPI == 1 ? NJT : 1][4][NS] = {};
            if constexpr (EPI == 1) {
#pragma unroll
                for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        gather(tc, XAXIS ? jt * 16 + lr : jt * 16 + M::row(lg, r), XAXIS ? M::row(lg, r) : lr,
                               old[jt][r]);
            }
#pragma unroll
            for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    emit(tc, XAXIS ? jt * 16 + lr : jt * 16 + M::row(lg, r), XAXIS ? M::row(lg, r) : lr,
                         (double)acc[jt][r], SYM == 2 ? (double)acc2[SYM == 2 ? jt : 0][r] : 0.0,
                         old[EPI == 1 ? jt : 0][r]);
            (void)acc2;
        }
    }
}

template <typename C, int PW, bool XAXIS, int EPI, typename TI, typename TO, int SYM>
static hipError_t panel_go(const TI* in, TO* out, const double* T, int n, int np, long nrows, long inner,
                           long ntiles, double alpha, hipStream_t st, const int* guard) {
    // the inverse split computes the outputs j < n / 2 (and their mirrors)
    const int ncols = SYM == 2 ? n / 2 : np;
    const int npanel = ncols / PW;
    if (npanel * PW != ncols) return hipErrorInvalidValue;
    const int kp = SYM == 1 ? n / 2 : (SYM == 2 ? n : 64 * ((np + 63) / 64));
    const size_t shm = panel_lds<C>(kp, PW);
    if (shm > 160 * 1024) return hipErrorInvalidValue;
    static std::atomic<bool> attr_set{false};       // set once; the attribute call is idempotent
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t e = hipFuncSetAttribute((const void*)k_xform_panel<C, PW, XAXIS, EPI, TI, TO, SYM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set.store(true, std::memory_order_release);
    }
    const long fit = (long)((160 * 1024) / shm);
    // 1, 2 or 4 blocks per compute unit (4 x 8 waves = 32 waves): a power of
    // two, so that halving below keeps a multiple of 8 npanel blocks
    const long per_cu = fit >= 4 ? 4 : (fit >= 2 ? 2 : 1);
    // persistent blocks: a multiple of 8 npanel, no more than the tiles need
    long blocks = 256 * per_cu;
    const long need = ((ntiles + kPanelWaves - 1) / kPanelWaves) * npanel;
    while (blocks > 8 * npanel && blocks / 2 >= need) blocks /= 2;
    hipLaunchKernelGGL((k_xform_panel<C, PW, XAXIS, EPI, TI, TO, SYM>), dim3((unsigned)blocks), dim3(kPanelThreads),
                       shm, st, in, out, T, n, np, npanel, nrows, inner, ntiles, alpha, guard);
    return hipGetLastError();
}

// panel width: the widest of 128 (64 in FP64), 64, 32 that divides np (the
// split transforms: n / 2)
template <typename C> static int panel_width(int np) {
    for (int pw : {128, 64, 32})
        if (pw <= PanelTraits<C>::PW && np % pw == 0) return pw;
    return 0;
}

template <typename C, bool XAXIS, int EPI, typename TI = double, typename TO = double>
static hipError_t panel_pw(int sym, const TI* in, TO* out, const double* T, int n, int np, long nrows, long inner,
                           long ntiles, double alpha, hipStream_t st, const int* guard) {
    if (sym == 1) {
        // the folding loads take a second set of registers: width 128 on the
        // x axis only (n / 2 is 64 or 128)
        if (EPI != 0) return hipErrorInvalidValue;
        // (in FP64 too: half as many panels re-read each line)
        if constexpr (XAXIS)
            if (n == 256) return panel_go<C, 128, XAXIS, EPI, TI, TO, 1>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
        return panel_go<C, 64, XAXIS, EPI, TI, TO, 1>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
    }
    if (sym == 2) {
        // two accumulator sets (even and odd modes): on the strided axis,
        // whose addressing takes more registers, at half the width
        if constexpr (XAXIS) {
            // (the update epilogue holds the old outputs too: width 64)
            if constexpr (PanelTraits<C>::PW >= 128 && EPI != 1)
                if (n == 256) return panel_go<C, 128, XAXIS, EPI, TI, TO, 2>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
            return panel_go<C, 64, XAXIS, EPI, TI, TO, 2>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
        } else {
            if constexpr (std::is_same<C, PanelF32>::value)
                if (n == 256) return panel_go<C, 64, XAXIS, EPI, TI, TO, 2>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
            return panel_go<C, 32, XAXIS, EPI, TI, TO, 2>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
        }
    }
    switch (panel_width<C>(np)) {
        case 32: return panel_go<C, 32, XAXIS, EPI, TI, TO, 0>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
        case 64: return panel_go<C, 64, XAXIS, EPI, TI, TO, 0>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
        case 128:
            if constexpr (PanelTraits<C>::PW >= 128)
                return panel_go<C, 128, XAXIS, EPI, TI, TO, 0>(in, out, T, n, np, nrows, inner, ntiles, alpha, st, guard);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

// io 0: double data; 2: float output (a forward transform's intermediate);
// 1: float input (an inverse transform's intermediate); float data only in
// the reduced precisions
template <typename C>
static hipError_t panel_x_epi(int sym, int epi, int io, const double* in, double* out, const double* T, int n,
                              int np, long lines, double alpha, hipStream_t st, const int* guard) {
    const long ntiles = (lines + 15) / 16;
    if (io == 0) {
        if (epi == 0) return panel_pw<C, true, 0>(sym, in, out, T, n, np, lines, 0, ntiles, alpha, st, guard);
        if (sym == 1) return hipErrorInvalidValue;
        if (epi == 1) return panel_pw<C, true, 1>(sym, in, out, T, n, np, lines, 0, ntiles, alpha, st, guard);
        return panel_pw<C, true, 2>(sym, in, out, T, n, np, lines, 0, ntiles, alpha, st, guard);
    }
    if constexpr (!std::is_same<C, PanelF64>::value) {
        if (io == 2) {
            if (epi != 0 || sym == 2) return hipErrorInvalidValue;
            return panel_pw<C, true, 0, double, float>(sym, in, (float*)out, T, n, np, lines, 0, ntiles, alpha, st,
                                                       guard);
        }
        if (io == 1) {
            if (sym == 1) return hipErrorInvalidValue;
            const float* fin = (const float*)in;
            if (epi == 0) return panel_pw<C, true, 0, float, double>(sym, fin, out, T, n, np, lines, 0, ntiles, alpha, st, guard);
            if (epi == 1) return panel_pw<C, true, 1, float, double>(sym, fin, out, T, n, np, lines, 0, ntiles, alpha, st, guard);
            return panel_pw<C, true, 2, float, double>(sym, fin, out, T, n, np, lines, 0, ntiles, alpha, st, guard);
        }
    }
    return hipErrorInvalidValue;
}

bool xform_panel_supported(int np) { return np >= 32 && np <= 256 && np % 32 == 0; }

bool xform_panel_split_supported(int n) { return n == 128 || n == 256; }

bool xform_panel_f32_io(int np) { return xform_panel_supported(np); }

hipError_t launch_xform_panel_x(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                                long lines, double alpha, hipStream_t st, const int* guard, int sym) {
    return launch_xform_panel_x_io(prec, epi, in, out, T, n, np, lines, alpha, st, guard, sym, 0);
}

hipError_t launch_xform_panel_x_io(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                                   long lines, double alpha, hipStream_t st, const int* guard, int sym, int io) {
    if (lines <= 0) return hipSuccess;
    if (!xform_panel_supported(np) || epi < 0 || epi > 2 || sym < 0 || sym > 2 || io < 0 || io > 2)
        return hipErrorInvalidValue;
    if (sym != 0 && !(xform_panel_split_supported(n) && np == n)) return hipErrorInvalidValue;
    if (prec == 0) return panel_x_epi<PanelF64>(sym, epi, io, in, out, T, n, np, lines, alpha, st, guard);
    if (prec == 1) return panel_x_epi<PanelF32>(sym, epi, io, in, out, T, n, np, lines, alpha, st, guard);
    if (prec == 2) return panel_x_epi<PanelBf16x3>(sym, epi, io, in, out, T, n, np, lines, alpha, st, guard);
    return hipErrorInvalidValue;
}

template <typename C>
static hipError_t panel_s_io(int sym, const double* in, double* out, const double* T, int n, int np, long inner,
                             long ntiles, hipStream_t st, const int* guard, int io_f32) {
    // float data: written by a forward transform, read by an inverse one
    if (io_f32 == 2) {
        if (sym == 2) return hipErrorInvalidValue;
        return panel_pw<C, false, 0, double, float>(sym, in, (float*)out, T, n, np, 0, inner, ntiles, 1.0, st, guard);
    }
    if (io_f32 == 1) {
        if (sym == 1) return hipErrorInvalidValue;
        return panel_pw<C, false, 0, float, double>(sym, (const float*)in, out, T, n, np, 0, inner, ntiles, 1.0, st,
                                                    guard);
    }
    if (io_f32 == 3) {
        // float on both sides (the intermediate of a reduced-precision transform)
        if constexpr (!std::is_same<C, PanelF64>::value)
            return panel_pw<C, false, 0, float, float>(sym, (const float*)in, (float*)out, T, n, np, 0, inner, ntiles,
                                                       1.0, st, guard);
        return hipErrorInvalidValue;
    }
    return panel_pw<C, false, 0>(sym, in, out, T, n, np, 0, inner, ntiles, 1.0, st, guard);
}

hipError_t launch_xform_panel_s(int prec, const double* in, double* out, const double* T, int n, int np, long nbatch,
                                long inner, hipStream_t st, const int* guard, int io_f32, int sym) {
    if (nbatch <= 0 || inner <= 0) return hipSuccess;
    if (!xform_panel_supported(np) || io_f32 < 0 || io_f32 > 3 || sym < 0 || sym > 2) return hipErrorInvalidValue;
    if (sym != 0 && !(xform_panel_split_supported(n) && np == n)) return hipErrorInvalidValue;
    const long ntiles = nbatch * ((inner + 15) / 16);
    if (prec == 0) return panel_s_io<PanelF64>(sym, in, out, T, n, np, inner, ntiles, st, guard, io_f32);
    if (prec == 1) return panel_s_io<PanelF32>(sym, in, out, T, n, np, inner, ntiles, st, guard, io_f32);
    if (prec == 2) return panel_s_io<PanelBf16x3>(sym, in, out, T, n, np, inner, ntiles, st, guard, io_f32);
    return hipErrorInvalidValue;
}

}  // namespace sth
