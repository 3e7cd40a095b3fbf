// C ABI of the slab solver: handle, device data, smoother, V-cycle, solve.
//
// The multigrid follows Section 3.1: damped block-Jacobi smoothing
//   u <- u + omega D^{-1}(f - L_h u),  D = diag(A_n),
// coarsening in time by combining two consecutive slabs (restriction
// P_t^T, prolongation P_t, the coarse slab operators are the Galerkin
// products, which equal a rediscretisation on the double-length slab with
// the finest SUPG parameter), V(nu_pre, nu_post) cycles, and an exact
// slab-wise forward substitution on the coarsest level.  D^{-1} is applied by
// eq. equ:ST:generalDecompA: spatial eigenbasis transforms (fast
// diagonalisation of the 1-D pencils), temporal eigenvector transform and
// shifted divide, inverse transforms.
#include <hip/hip_runtime.h>
#include <atomic>
#include <chrono>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sth.h"
#include "kernels.hpp"
#include "setup.hpp"
#include "solve_async.hpp"

using namespace sth;

static thread_local std::string g_err;

// squared norms on the device and their mapped host copies: [0] exact
// residual, [1] right-hand side, then three cycle slots of three sums each
// (eigenbasis residual, its lower and its upper mode-weighted sums; slots 0
// and 1 alternate between cycles, slot 2 is the initial pass of a
// speculative solve), then the outer residual and right-hand side of a
// mixed-precision solve
constexpr int kNormSlots = 14;
constexpr int slot_base(int slot) { return 2 + 3 * slot; }
constexpr int kMixR = 11, kMixF = 12;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(STH_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct sth_handle {
    Setup S;
    int dim = 2, n = 0, np = 0, Nt = 0, p = 0, L = 0;
    long Nx = 0;
    long Nxe = 0;                       // modes per time row of an eigenbasis vector (eig_modes)
    // the spatial modes are ordered [even | odd] under the reflection
    // i -> n-1-i and the per-axis transforms use the split kernels
    bool split = false;
    double omega = 0.5;
    int nu_pre = 1, nu_post = 1;
    int prec = 0;                       // sth_prec of the spatial transforms
    std::vector<long> lev_S;            // slabs per level
    std::vector<TimeOp> ops;
    std::vector<TimeMix> mixes;
    Transfer tr{};
    // device data
    double* Tf = nullptr;               // np x np, U padded  (forward: r^ = U^T r)
    double* Ti = nullptr;               // np x np, U^T padded (inverse: z = U z^)
    double* mu1 = nullptr;
    double* M1b = nullptr;
    double* K1b = nullptr;
    double* dktmt = nullptr;            // per level: K_t then M_t (kNt x kNt each)
    std::vector<double*> lu, lf;        // per level >= 1: iterate and right-hand side
    // iteration in the spatial eigenbasis (iterate_basis = 1)
    int basis = 0;
    double* Cf = nullptr;               // np x np, C = M_1 U padded (C = U^{-T})
    double* Ci = nullptr;               // np x np, C^T padded
    double* Gf = nullptr;               // np x np, G = C^T C padded (2-D, np <= 96)
    double* e0 = nullptr;               // f^ on level 0
    double* e1 = nullptr;               // u^ on level 0 (ping-pong with e2)
    double* e2 = nullptr;
    double* e3 = nullptr;               // third level-0 iterate buffer of the fused cycle close
    bool fuse_close = false;            // post-smoothing of level 0 fused into the cycle-end pass
    bool fuse_tail = false;             // the two coarsest levels in one pass (k_eig_coarse_tail)
    bool fuse_tail3 = false;            // the three coarsest levels in one pass (k_eig_coarse_tail3)
    TimeMix* dmix = nullptr;            // per level slab inverse in device memory
    bool defer_close = false;           // set by a solve iteration: level 0 leaves its post-smoothing
    const double* pending_ec = nullptr; // coarse correction waiting for the fused cycle close
    // The solve loop's fused cycle closes do not store the cycle's result
    // (level-0 buffer dst): it is formed from the close's inputs (the
    // pre-smoothed buffer c and the coarse correction ec, which stay intact
    // until the next cycle runs) only when it is read (form_result).
    // A zero initial guess is likewise left unwritten (zero): buffer dst is
    // filled with zeros when read, where the device flag zguard is 0 (always
    // without one); the initial pass reads that flag instead of the buffer.
    struct Unformed {
        bool on = false;
        int c = 0, dst = 0;
        const double* ec = nullptr;
        bool zero = false;
        const int* zguard = nullptr;
    };
    Unformed unformed;
    bool lazy_close = false;            // set by the solve loop around its cycles
    const int* zero_in = nullptr;       // device flag of an unwritten zero guess (Unformed::zero)
    int pre_idx = 1;                    // level-0 buffer of the pre-smoothed iterate
    std::vector<double*> lu2;           // ping-pong partner of lu on levels >= 1
    // FP32 storage of the eigenbasis vectors (the inner solves of the mixed
    // precision form): e0..e3 and the coarse-level eu, ef, eu2 hold floats
    // (the pointers then address float data; arithmetic stays FP64)
    bool f32 = false;
    std::vector<double*> eu, ef, eu2;
    std::vector<int> ecur;              // which buffer of the pair holds u^ per level
    bool presmoothed = false;           // level-0 buffer pre_idx holds u^ after one smoothing step
                                        // and lf[1] the restriction of its residual
    double* cpartial = nullptr;         // per-block partial sums of the cycle-end pass
    long n_cpartial = 0;
    // FGMRES workspace (allocated by the first sth_solve_fgmres)
    int k_alloc = 0;                    // restart length the workspace holds
    double* kv = nullptr;               // (restart+1) Krylov vectors
    double* kz = nullptr;               // restart preconditioned vectors
    double* kc = nullptr;               // kMaxKrylov coefficients / dot products
    double* kpart = nullptr;            // 1024 x kMaxKrylov partial sums
    double* khost = nullptr;            // pinned copy of kc
    double nb_lo = 0.0;                 // ||(I (x) C) r^||^2 >= nb_lo ||r^||^2
    double nb_hi = 0.0;                 // ||(I (x) C) r^||^2 <= nb_hi ||r^||^2
    double* vw = nullptr;               // per axis and 1-D mode: G_jj and sum_k |G_jk| (G = C^T C)
    bool wsum_valid = false;            // the norm slots hold the mode-weighted residual sums
    double* buf0 = nullptr;
    double* buf1 = nullptr;
    // coarsening in space (Section 4.4): the transition below the last
    // level of this handle halves the spatial mesh as well; the levels from
    // there on belong to `child`, the problem on the halved mesh
    sth_handle* child = nullptr;
    int n_c = 0;                        // interior functions per axis of the child's mesh
    int rW = 0, pW = 0;                 // band widths of P_x^T and P_x
    int* rj0 = nullptr;                 // P_x^T: first fine function of each coarse one
    double* rco = nullptr;              //   and its rW coefficients
    int* pj0 = nullptr;                 // P_x: first coarse function of each fine one
    double* pco = nullptr;              //   and its pW coefficients
    double* cf = nullptr;               // right-hand side and iterate of the child's finest level
    double* cu = nullptr;
    // MinRes slab inverse of the smoother (minres_iters > 0): per level the
    // mixing into the temporal blocks (W, the pair rows scaled as in
    // Theorem 3.10), back (V, the second row of a pair negated), the 2x2
    // operators and the preconditioner's per-row shifts; level-0-sized
    // vectors v_{j-1}, v_j, v_{j+1}, z_j, z_{j+1}, w_{j-1}, w_{j-2}, y and the
    // per-system scalars
    int minres = 0;
    std::vector<TimeRowMix> mr_win, mr_vout;
    std::vector<PairOps> mr_ops;
    std::vector<PinvRows> mr_pinv;
    double* mr[8] = {};
    double* mrst = nullptr;
    double* partial = nullptr;
    double* dnorm = nullptr;            // squared norms (layout at kNormSlots)
    double* hnorm = nullptr;            // pinned, mapped, coherent host copies of dnorm
    double* hnorm_dev = nullptr;        // device address of hnorm
    // timing
    bool timing = false;
    unsigned timing_mask = 0;
    int timing_level = -1;              // record only launches on this level (-1: all)
    int tlev = 0;                       // level of the launches being enqueued
    struct Rec { int cls; hipEvent_t a, b; double flops, bytes; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    // graph of one solve iteration (V-cycle, residual, norm, scalar read)
    bool use_graph = false;
    bool capturing = false;
    // two cached graphs: the fused cycle close alternates its level-0
    // buffers, so consecutive iterations start from two different states
    struct GraphEntry {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        const double* f = nullptr;
        double* u = nullptr;
        unsigned mask = 0;
        int key = -1;                   // level-0 buffer state at entry
        int ecur0_after = 0, pre_after = 1, slot_after = 0;
        bool presm_after = false;
        Unformed unf_after;
        std::vector<Rec> recs;          // timed launches inside the graph
        long last_used = 0;
    } gent[2];
    long graph_clock = 0;
    GraphEntry* glast = nullptr;        // entry of the last replay (its timings)
    bool allow_capture = true;          // cleared by the serving loop while another thread allocates
    bool graph_launched = false;        // the last enqueued iteration was a graph replay
    std::vector<Rec> grecs;             // timed launches of the graph being captured
    double gms[STH_K_COUNT] = {0}, gfl[STH_K_COUNT] = {0}, gby[STH_K_COUNT] = {0};
    int gcnt[STH_K_COUNT] = {0};
    // state of the solve in progress (sth_solve and the serving loop)
    // level-0 buffer state after an enqueued cycle, and its norm slot
    struct Snap {
        int ecur0 = 0, pre_idx = 1;
        bool presmoothed = false;
        int slot = 0;
        int seqv = 0;                   // completion mark of the cycle's final sum
        Unformed unf;
    };
    struct SolveState {
        const double* f = nullptr;
        double* u = nullptr;
        hipStream_t st = nullptr;
        double rtol = 0.0, fn = 1.0, rn = 0.0, prev = 0.0;
        int maxit = 0, it = 0, growth = 0;
        // 0 initial norms enqueued, 1 iterating, 2 result enqueued, 3 exact
        // B-spline norm of the current eigenbasis iterate enqueued, 4 initial
        // norms enqueued with the first cycles behind them (speculation)
        int phase = 0;
        // speculation: the cycle waited for (a) and the guarded one behind it (b)
        bool spec = false;
        int pend = 0;
        bool drain = false;
        Snap a, b, s0;                  // s0: state after the initial norms
        // the mapping of the result into u was enqueued behind the exact norm
        // (fin_always: unguarded, as the cycle count or growth ends the solve)
        bool fin_enq = false, fin_always = false;
        hipEvent_t ev_a = nullptr, ev_b = nullptr;
        // inner solve of a mixed-precision solve: zero initial guess, ||f||
        // known, transforms in precision tprec, no exact B-spline norm (the
        // lower bound decides), the result added into u
        bool inner = false;
        bool inner_store = false;       // the inner result is stored into u (u was zero), not added
        int tprec = STH_FP64;
    } sv;
    // Mixed-precision solve (eigenbasis iteration with reduced-precision
    // transforms): FP64 defect correction around inner eigenbasis solves
    struct Mixed {
        bool on = false;
        const double* f = nullptr;
        double* u = nullptr;
        hipStream_t st = nullptr;
        double rtol = 0.0, fn = 1.0, rn = 0.0, prev = 0.0;
        int maxit = 0, it = 0, outer = 0, growth = 0;
        int phase = 0;                  // 0 outer residual norm enqueued, 1 inner solve running, 2 done,
                                        // 3 ||f|| and whether u is nonzero enqueued
    } mx;
    // speculative cycles (eigenbasis, fused cycle close)
    bool speculate = true;
    const int* guard = nullptr;         // guard of the launches of the cycle being enqueued
    int* dgo = nullptr;                 // per norm slot: continuation flag of the cycle (device);
                                        // [2]: the final exact norm ends the solve; [3]: the
                                        // initial pass of a speculative solve; [4]: the initial
                                        // guess of the solve has a nonzero entry; [5]: always 0
    int* hflag = nullptr;               // its mapped host copy
    int* hflag_dev = nullptr;
    double* dthr = nullptr;             // (rtol ||f||)^2 and rtol ||f|| of the solve in progress (device)
    int last_slot = 0;                  // norm slot of the last enqueued cycle end
    bool first_flag = false;            // the initial residual pass sets its own flag (dgo[3])
    bool first_guard = false;           // the next cycle is guarded by it
    hipEvent_t evring[4] = {nullptr, nullptr, nullptr, nullptr};
    int evnext = 0;
    hipEvent_t wait_ev = nullptr;       // event the caller waits for before solve_continue
    // or (wait_slot >= 0) the completion mark wait_seq in hseq[wait_slot]:
    // the blocking solve with eager launches polls mapped memory instead of
    // recording an event per cycle (an event record leaves the GPU idle for
    // a few microseconds at every cycle boundary)
    int* hseq = nullptr;                // mapped, coherent: per norm slot, last completion mark
    int* hseq_dev = nullptr;
    int seq_counter = 0, last_seq = 0;
    int wait_slot = -1, wait_seq = 0;
    bool want_poll = false, poll_seq = false;
};

static void drop_graph_entry(sth_handle::GraphEntry& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = sth_handle::GraphEntry{};
}

static void drop_graph(sth_handle* h) {
    for (auto& g : h->gent) drop_graph_entry(g);
    h->glast = nullptr;
    h->grecs.clear();
}

static long slab_len(const sth_handle* h) { return (long)h->Nt * h->Nx; }
// slab length of an eigenbasis vector (time rows padded to eig_modes)
static long eslab_len(const sth_handle* h) { return (long)h->Nt * h->Nxe; }

// ---------------------------------------------------------------------------
// timing helpers
// ---------------------------------------------------------------------------
struct Timed {
    sth_handle* h;
    int cls;
    double flops, bytes;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(sth_handle* hh, int c, double fl, double by, hipStream_t s) : h(hh), cls(c), flops(fl), bytes(by), st(s) {
        if (!h->timing || !((h->timing_mask >> c) & 1u)) return;
        if (h->timing_level >= 0 && h->tlev != h->timing_level) return;
        if (h->pool_used + 2 > h->pool.size()) {
            for (int i = 0; i < 256; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                h->pool.push_back(e);
            }
        }
        a = h->pool[h->pool_used++];
        b = h->pool[h->pool_used++];
        (void)hipEventRecord(a, st);
    }
    ~Timed() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        // inside a graph capture the pair becomes two event-record nodes that
        // fire on every replay; their times are summed after each replay
        (h->capturing ? h->grecs : h->recs).push_back({cls, a, b, flops, bytes});
    }
};

// ---------------------------------------------------------------------------
// building blocks
// ---------------------------------------------------------------------------
static int residual(sth_handle* h, int lvl, const double* f, const double* u, double* r, long s0, long ns,
                    double sign, hipStream_t st) {
    h->tlev = lvl;
    double dof = (double)ns * slab_len(h);
    int B = 2 * h->p + 1;
    double flops = dof * ((h->dim == 2 ? 10.0 : 16.0) * B + 4.0 * h->Nt + 2.0);
    double bytes = dof * (f ? 24.0 : 16.0);
    Timed tm(h, STH_K_RESIDUAL, flops, bytes, st);
    HIPCHK(launch_residual(h->dim, h->Nt, h->p, h->n, h->M1b, h->K1b, h->ops[lvl],
                           h->dktmt + (size_t)lvl * 2 * kNt * kNt, f, u, r, s0, ns, sign, st));
    return STH_OK;
}

// Split form of a per-axis transform with matrix T: 1 for the forward
// matrices (U, C = M_1 U: out = T^T in), 2 for the inverse ones (their
// transposes), 0 without the even/odd mode order
static int split_of(const sth_handle* h, const double* T) {
    if (!h->split) return 0;
    if (T == h->Tf || (h->Cf && T == h->Cf)) return 1;
    if (T == h->Ti || (h->Ci && T == h->Ci)) return 2;
    return 0;
}

// per-axis transforms in the precision `prec` (sth_prec); the split forms
// take n / 2 multiply-adds per output instead of n
// io (reduced precisions): 2 float output, 1 float input
static int xform_x(sth_handle* h, int prec, int epi, const double* in, double* out, const double* T, long lines,
                   double alpha, hipStream_t st, const int* guard = nullptr, int io = 0) {
    const double dof = (double)lines * h->n;
    const int sym = split_of(h, T);
    Timed tm(h, STH_K_XFORM_X, (sym ? 1.0 : 2.0) * h->n * dof, dof * ((epi == 1 ? 24.0 : 16.0) - (io ? 4.0 : 0.0)),
             st);
    HIPCHK(launch_xform_x(prec, epi, in, out, T, h->n, h->np, lines, alpha, st, guard, sym, io));
    return STH_OK;
}

static int xform_s(sth_handle* h, int prec, const double* in, double* out, const double* T, long nbatch,
                   long inner, hipStream_t st, const int* guard = nullptr, int io_f32 = 0) {
    const double dof = (double)nbatch * h->n * inner;
    const int sym = split_of(h, T);
    Timed tm(h, STH_K_XFORM_S, (sym ? 1.0 : 2.0) * h->n * dof, (io_f32 == 3 ? 8.0 : (io_f32 ? 12.0 : 16.0)) * dof, st);
    HIPCHK(launch_xform_s(prec, in, out, T, h->n, h->np, nbatch, inner, st, guard, io_f32, sym));
    return STH_OK;
}

// u (mode 1: +=, 2: =) omega * D^{-1} in, on slabs [s0, s0+ns) of level lvl.
// `in` may alias buf1 but not buf0.
static int slab_inverse(sth_handle* h, int lvl, const double* in, double* u, int epi, double alpha, long s0,
                        long ns, hipStream_t st, bool fwdsub = false) {
    h->tlev = lvl;
    long off = s0 * slab_len(h);
    in += off;
    u += off;
    const long n = h->n;
    const long rows = ns * h->Nt;           // time rows
    double* b0 = h->buf0 + off;
    double* b1 = h->buf1 + off;
    int rc;
    if (h->dim == 2 && xform2d_supported(h->np)) {
        double dof = (double)ns * slab_len(h);
        {
            Timed tm(h, STH_K_XFORM_2D, 4.0 * h->n * dof, 16.0 * dof, st);
            if (h->prec == STH_BF16X3)
                HIPCHK(launch_xform2d_bf16x3(0, in, b0, h->Ti, h->n, h->np, rows, 1.0, st));
            else
                HIPCHK(launch_xform2d(h->prec, 0, 0, in, b0, h->Tf, h->n, h->np, rows, 1.0, st));
        }
        {
            Timed tm(h, STH_K_TIMEMIX, dof * (4.0 * h->Nt + 4.0), 16.0 * dof, st);
            HIPCHK(launch_timemix(2, h->Nt, h->mixes[lvl], h->mu1, h->n, 0, b0, b1, ns, fwdsub, st));
        }
        {
            Timed tm(h, STH_K_XFORM_2D, 4.0 * h->n * dof, (epi == 1 ? 24.0 : 16.0) * dof, st);
            if (h->prec == STH_BF16X3)
                HIPCHK(launch_xform2d_bf16x3(epi, b1, u, h->Tf, h->n, h->np, rows, alpha, st));
            else
                HIPCHK(launch_xform2d(h->prec, 1, epi, b1, u, h->Tf, h->n, h->np, rows, alpha, st));
        }
    } else if (h->dim == 2) {
        const int pr = h->prec;
        if ((rc = xform_x(h, pr, 0, in, b0, h->Tf, rows * n, 1.0, st))) return rc;
        if ((rc = xform_s(h, pr, b0, b1, h->Tf, rows, n, st))) return rc;
        {
            double dof = (double)ns * slab_len(h);
            Timed tm(h, STH_K_TIMEMIX, dof * (4.0 * h->Nt + 4.0), 16.0 * dof, st);
            HIPCHK(launch_timemix(2, h->Nt, h->mixes[lvl], h->mu1, h->n, 0, b1, b0, ns, fwdsub, st));
        }
        if ((rc = xform_s(h, pr, b0, b1, h->Ti, rows, n, st))) return rc;
        if ((rc = xform_x(h, pr, epi, b1, u, h->Ti, rows * n, alpha, st))) return rc;
    } else {
        const int pr = h->prec;
        if ((rc = xform_x(h, pr, 0, in, b0, h->Tf, rows * n * n, 1.0, st))) return rc;
        if ((rc = xform_s(h, pr, b0, b1, h->Tf, rows * n, n, st))) return rc;      // y
        if ((rc = xform_s(h, pr, b1, b0, h->Tf, rows, n * n, st))) return rc;      // z
        {
            double dof = (double)ns * slab_len(h);
            Timed tm(h, STH_K_TIMEMIX, dof * (4.0 * h->Nt + 4.0), 16.0 * dof, st);
            HIPCHK(launch_timemix(3, h->Nt, h->mixes[lvl], h->mu1, h->n, 0, b0, b1, ns, fwdsub, st));
        }
        if ((rc = xform_s(h, pr, b1, b0, h->Ti, rows, n * n, st))) return rc;      // z
        if ((rc = xform_s(h, pr, b0, b1, h->Ti, rows * n, n, st))) return rc;      // y
        if ((rc = xform_x(h, pr, epi, b1, u, h->Ti, rows * n * n, alpha, st))) return rc;
    }
    return STH_OK;
}

// out = P^{-1} in per time row: the spatial transforms of the slab inverse
// around a per-row scale / (mu + shift) in the eigenbasis (the exact inverse
// of K_x + shift M_x, times scale); buf0 and buf1 are the work vectors
static int pinv_apply(sth_handle* h, int lvl, const double* in, double* out, long ns, hipStream_t st) {
    h->tlev = lvl;
    const long n = h->n, rows = ns * h->Nt;
    double* b0 = h->buf0;
    double* b1 = h->buf1;
    const double dof = (double)ns * slab_len(h);
    int rc;
    auto scale = [&](double* t) -> int {
        Timed tm(h, STH_K_TIMEMIX, 2.0 * dof, 16.0 * dof, st);
        HIPCHK(launch_pinv_scale(t, ns, h->Nt, h->Nx, h->dim, h->mu1, h->n, h->mr_pinv[lvl], st));
        return STH_OK;
    };
    if (h->dim == 2 && xform2d_supported(h->np)) {
        {
            Timed tm(h, STH_K_XFORM_2D, 4.0 * h->n * dof, 16.0 * dof, st);
            if (h->prec == STH_BF16X3)
                HIPCHK(launch_xform2d_bf16x3(0, in, b0, h->Ti, h->n, h->np, rows, 1.0, st));
            else
                HIPCHK(launch_xform2d(h->prec, 0, 0, in, b0, h->Tf, h->n, h->np, rows, 1.0, st));
        }
        if ((rc = scale(b0))) return rc;
        Timed tm(h, STH_K_XFORM_2D, 4.0 * h->n * dof, 16.0 * dof, st);
        if (h->prec == STH_BF16X3)
            HIPCHK(launch_xform2d_bf16x3(0, b0, out, h->Tf, h->n, h->np, rows, 1.0, st));
        else
            HIPCHK(launch_xform2d(h->prec, 1, 0, b0, out, h->Tf, h->n, h->np, rows, 1.0, st));
    } else if (h->dim == 2) {
        const int pr = h->prec;
        if ((rc = xform_x(h, pr, 0, in, b0, h->Tf, rows * n, 1.0, st))) return rc;
        if ((rc = xform_s(h, pr, b0, b1, h->Tf, rows, n, st))) return rc;
        if ((rc = scale(b1))) return rc;
        if ((rc = xform_s(h, pr, b1, b0, h->Ti, rows, n, st))) return rc;
        if ((rc = xform_x(h, pr, 0, b0, out, h->Ti, rows * n, 1.0, st))) return rc;
    } else {
        const int pr = h->prec;
        if ((rc = xform_x(h, pr, 0, in, b0, h->Tf, rows * n * n, 1.0, st))) return rc;
        if ((rc = xform_s(h, pr, b0, b1, h->Tf, rows * n, n, st))) return rc;      // y
        if ((rc = xform_s(h, pr, b1, b0, h->Tf, rows, n * n, st))) return rc;      // z
        if ((rc = scale(b0))) return rc;
        if ((rc = xform_s(h, pr, b0, b1, h->Ti, rows, n * n, st))) return rc;      // z
        if ((rc = xform_s(h, pr, b1, b0, h->Ti, rows * n, n, st))) return rc;      // y
        if ((rc = xform_x(h, pr, 0, b0, out, h->Ti, rows * n * n, 1.0, st))) return rc;
    }
    return STH_OK;
}

// u = alpha A^{-1} in (epi 2) or u += alpha A^{-1} in (epi 1) on the ns slabs
// of level lvl, A^{-1} through the temporal eigen form: g = W in (pair rows
// scaled by |b2|, |b1|), the real rows' systems solved exactly by P^{-1},
// each pair's symmetric system of Theorem 3.10 by h->minres MinRes
// iterations preconditioned by P (all (slab, pair) systems together, each
// with its own scalars), then u (+)= alpha V y with the second row of each
// pair negated (the substitution of the theorem).  `in` may be buf1.
static int minres_slab_inverse(sth_handle* h, int lvl, const double* in, double* u, int epi, double alpha, long ns,
                               hipStream_t st) {
    h->tlev = lvl;
    const int nt = h->Nt, npairs = h->mr_ops[lvl].npairs;
    const long nx = h->Nx, nsys = ns * npairs;
    const double dof = (double)ns * slab_len(h);
    double *vp = h->mr[0], *vc = h->mr[1], *vn = h->mr[2], *zc = h->mr[3], *zn = h->mr[4];
    double *w1 = h->mr[5], *w2 = h->mr[6], *y = h->mr[7];
    double* q = h->buf0;
    int rc;
    {
        Timed tm(h, STH_K_TIMEMIX, 2.0 * nt * dof, 16.0 * dof, st);
        HIPCHK(launch_time_mix(in, vc, h->mr_win[lvl], ns, nt, nx, 0, 1.0, st));
    }
    if ((rc = pinv_apply(h, lvl, vc, y, ns, st))) return rc;
    if (npairs > 0) {
        h->tlev = lvl;
        const double pdof = (double)nsys * 2 * nx;
        {
            Timed tm(h, STH_K_OTHER, 0.0, 40.0 * pdof, st);
            HIPCHK(launch_pair_split(y, zc, w1, w2, vp, ns, nt, npairs, nx, st));
            HIPCHK(launch_pair_dot(vc, zc, h->mrst, 1, ns, nt, npairs, nx, st));
            HIPCHK(launch_minres_init(h->mrst, nsys, st));
        }
        for (int it = 0; it < h->minres; ++it) {
            h->tlev = lvl;
            {
                const double st_pts = std::pow(2.0 * h->p + 1.0, h->dim);
                Timed tm(h, STH_K_MINRES, pdof * 4.0 * st_pts, 16.0 * pdof, st);
                HIPCHK(launch_pair_apply(h->dim, zc, q, h->M1b, h->K1b, h->n, h->p, ns, nt, h->mr_ops[lvl], st));
            }
            {
                Timed tm(h, STH_K_OTHER, 8.0 * pdof, 56.0 * pdof, st);
                HIPCHK(launch_pair_dot(q, zc, h->mrst, 0, ns, nt, npairs, nx, st));
                HIPCHK(launch_lanczos(q, vc, vp, vn, h->mrst, ns, nt, npairs, nx, st));
            }
            if ((rc = pinv_apply(h, lvl, vn, zn, ns, st))) return rc;
            h->tlev = lvl;
            {
                Timed tm(h, STH_K_OTHER, 8.0 * pdof, 56.0 * pdof, st);
                HIPCHK(launch_pair_dot(vn, zn, h->mrst, 1, ns, nt, npairs, nx, st));
                HIPCHK(launch_minres_scalars(h->mrst, nsys, st));
                HIPCHK(launch_minres_update(zc, w1, w2, y, h->mrst, ns, nt, npairs, nx, st));
            }
            std::swap(w1, w2);          // w_{j-1} <- w_j, w_{j-2} <- w_{j-1}
            double* t = vp;             // v_{j-1} <- v_j, v_j <- v_{j+1}
            vp = vc;
            vc = vn;
            vn = t;
            std::swap(zc, zn);
        }
    }
    Timed tm(h, STH_K_TIMEMIX, 2.0 * nt * dof, (epi == 1 ? 24.0 : 16.0) * dof, st);
    HIPCHK(launch_time_mix(y, u, h->mr_vout[lvl], ns, nt, nx, epi == 1 ? 1 : 0, alpha, st));
    return STH_OK;
}

// one damped block-Jacobi step on level lvl; zero_guess: u is taken as 0
static int smooth_step(sth_handle* h, int lvl, const double* f, double* u, bool zero_guess, hipStream_t st) {
    long ns = h->lev_S[lvl];
    if (zero_guess)
        return h->minres ? minres_slab_inverse(h, lvl, f, u, 2, h->omega, ns, st)
                         : slab_inverse(h, lvl, f, u, 2, h->omega, 0, ns, st);
    int rc = residual(h, lvl, f, u, h->buf1, 0, ns, 1.0, st);
    if (rc) return rc;
    return h->minres ? minres_slab_inverse(h, lvl, h->buf1, u, 1, h->omega, ns, st)
                     : slab_inverse(h, lvl, h->buf1, u, 1, h->omega, 0, ns, st);
}

// exact solve of the coarsest level: slab-wise forward substitution
//   u_1 = A^{-1} f_1,  u_m = A^{-1}(f_m + B u_{m-1})   (eq. equ_linear_system)
// carried out in the spatial eigenbasis, where A = K_t (x) I + M_t (x) diag(mu)
// and B = N_t (x) I: forward transforms of all slabs, the coupled slabs of
// every spatial mode solved parallel in time (a scalar recurrence carries the
// coupling), inverse transforms.  u is overwritten.
static int coarse_solve(sth_handle* h, int lvl, const double* f, double* u, hipStream_t st) {
    long S = h->lev_S[lvl];
    if (S == 1) return slab_inverse(h, lvl, f, u, 2, 1.0, 0, 1, st);
    return slab_inverse(h, lvl, f, u, 2, 1.0, 0, S, st, /*fwdsub=*/true);
}

static int restrict_lvl(sth_handle* h, int lvl, const double* r, double* rc, hipStream_t st) {
    h->tlev = lvl;
    long Sc = h->lev_S[lvl + 1];
    double dof = (double)Sc * slab_len(h);
    Timed tm(h, STH_K_RESTRICT, dof * 4.0 * h->Nt, dof * 24.0, st);
    HIPCHK(launch_restrict(h->Nt, h->tr, r, rc, Sc, h->Nx, st));
    return STH_OK;
}

// u += (P_t (x) I) e on the slab pairs of level lvl; row_len is the length
// of a time row: h->Nx for B-spline coefficient vectors, h->Nxe for
// eigenbasis vectors (their rows are padded)
static int prolong_lvl(sth_handle* h, int lvl, const double* e, double* u, hipStream_t st, long row_len) {
    h->tlev = lvl;
    long Sc = h->lev_S[lvl + 1];
    double dof = (double)Sc * slab_len(h);
    Timed tm(h, STH_K_PROLONG, dof * 4.0 * h->Nt, dof * 40.0, st);
    HIPCHK(launch_prolong(h->Nt, h->tr, e, u, Sc, row_len, st));
    return STH_OK;
}

// Space-time restriction from the last level of h to the child's finest
// level: r_c = (P_t^T (x) P_x^T (x) .. (x) P_x^T) on each slab pair, in time
// first (into buf0), then along x, y (and z), alternating buf1 and buf0.
// Neither r nor rc may be buf0 or buf1 of h, except r == buf1.
static int restrict_space(sth_handle* h, const double* r, double* rc, hipStream_t st) {
    const int lvl = h->L - 1;
    h->tlev = lvl;
    const long Sc = h->child->lev_S[0];
    const long nf = h->n, nc = h->n_c, rows = Sc * h->Nt;
    const double dof = (double)Sc * slab_len(h);
    Timed tm(h, STH_K_RESTRICT, dof * 4.0 * h->Nt + dof * 2.0 * h->rW * (h->dim == 2 ? 1.5 : 1.75),
             dof * 24.0, st);
    HIPCHK(launch_restrict(h->Nt, h->tr, r, h->buf0, Sc, h->Nx, st));
    if (h->dim == 2) {
        HIPCHK(launch_band_axis(h->buf0, h->buf1, rows * nf, nf, nc, 1, h->rj0, h->rco, h->rW, st));     // x
        HIPCHK(launch_band_axis(h->buf1, rc, rows, nf, nc, nc, h->rj0, h->rco, h->rW, st));               // y
    } else {
        HIPCHK(launch_band_axis(h->buf0, h->buf1, rows * nf * nf, nf, nc, 1, h->rj0, h->rco, h->rW, st));  // x
        HIPCHK(launch_band_axis(h->buf1, h->buf0, rows * nf, nf, nc, nc, h->rj0, h->rco, h->rW, st));      // y
        HIPCHK(launch_band_axis(h->buf0, rc, rows, nf, nc, nc * nc, h->rj0, h->rco, h->rW, st));           // z
    }
    return STH_OK;
}

// u += (P_t (x) P_x (x) .. (x) P_x) e on the slab pairs of the last level of h
// (e on the child's finest level): along z, y, x into the buffers, then the
// time prolongation adds into u.  Neither e nor u may be buf0 or buf1 of h.
static int prolong_space(sth_handle* h, const double* e, double* u, hipStream_t st) {
    const int lvl = h->L - 1;
    h->tlev = lvl;
    const long Sc = h->child->lev_S[0];
    const long nf = h->n, nc = h->n_c, rows = Sc * h->Nt;
    const double dof = (double)Sc * slab_len(h);
    Timed tm(h, STH_K_PROLONG, dof * 4.0 * h->Nt + dof * 2.0 * h->pW * 2.0, dof * 40.0, st);
    const double* fine;
    if (h->dim == 2) {
        HIPCHK(launch_band_axis(e, h->buf0, rows, nc, nf, nc, h->pj0, h->pco, h->pW, st));                 // y
        HIPCHK(launch_band_axis(h->buf0, h->buf1, rows * nf, nc, nf, 1, h->pj0, h->pco, h->pW, st));       // x
        fine = h->buf1;
    } else {
        HIPCHK(launch_band_axis(e, h->buf0, rows, nc, nf, nc * nc, h->pj0, h->pco, h->pW, st));            // z
        HIPCHK(launch_band_axis(h->buf0, h->buf1, rows * nf, nc, nf, nc, h->pj0, h->pco, h->pW, st));      // y
        HIPCHK(launch_band_axis(h->buf1, h->buf0, rows * nf * nf, nc, nf, 1, h->pj0, h->pco, h->pW, st));  // x
        fine = h->buf0;
    }
    HIPCHK(launch_prolong(h->Nt, h->tr, fine, u, Sc, h->Nx, st));
    return STH_OK;
}

static int vcycle_lvl(sth_handle* h, int lvl, const double* f, double* u, bool zero_guess, hipStream_t st);

// the coarse-grid correction below the last level of h: V-cycle of the
// child from a zero guess (its exact solve when it has one level)
static int child_cycle(sth_handle* c, const double* f, double* u, hipStream_t st) {
    if (c->L == 1 && !c->child) return coarse_solve(c, 0, f, u, st);
    return vcycle_lvl(c, 0, f, u, true, st);
}

static int vcycle_lvl(sth_handle* h, int lvl, const double* f, double* u, bool zero_guess, hipStream_t st) {
    h->tlev = lvl;
    int rc;
    if (lvl == h->L - 1 && !h->child) {
        if (lvl > 0) return coarse_solve(h, lvl, f, u, st);      // zero initial guess on coarse levels
        // a single level: correct the iterate, u += L^{-1}(f - L u), so that
        // an inexact (reduced-precision) forward substitution still converges
        const long S = h->lev_S[0];
        if ((rc = residual(h, 0, f, u, h->buf1, 0, S, 1.0, st))) return rc;
        return slab_inverse(h, 0, h->buf1, u, 1, 1.0, 0, S, st, /*fwdsub=*/S > 1);
    }
    long ns = h->lev_S[lvl];
    if (zero_guess && h->nu_pre == 0) {
        Timed tm(h, STH_K_OTHER, 0, 8.0 * ns * slab_len(h), st);
        HIPCHK(launch_fill(u, ns * slab_len(h), 0.0, st));
        zero_guess = false;
    }
    for (int i = 0; i < h->nu_pre; ++i) {
        if ((rc = smooth_step(h, lvl, f, u, zero_guess && i == 0, st))) return rc;
    }
    if ((rc = residual(h, lvl, f, u, h->buf1, 0, ns, 1.0, st))) return rc;
    if (lvl == h->L - 1) {
        // coarsening in space and time: the child's hierarchy below
        if ((rc = restrict_space(h, h->buf1, h->cf, st))) return rc;
        if ((rc = child_cycle(h->child, h->cf, h->cu, st))) return rc;
        h->tlev = lvl;
        if ((rc = prolong_space(h, h->cu, u, st))) return rc;
    } else {
        if ((rc = restrict_lvl(h, lvl, h->buf1, h->lf[lvl + 1], st))) return rc;
        if ((rc = vcycle_lvl(h, lvl + 1, h->lf[lvl + 1], h->lu[lvl + 1], true, st))) return rc;
        if ((rc = prolong_lvl(h, lvl, h->lu[lvl + 1], u, st, h->Nx))) return rc;
    }
    for (int i = 0; i < h->nu_post; ++i) {
        if ((rc = smooth_step(h, lvl, f, u, false, st))) return rc;
    }
    return STH_OK;
}

static int norm2_dev(sth_handle* h, const double* v, long len, hipStream_t st) {
    h->tlev = 0;
    Timed tm(h, STH_K_NORM, 2.0 * len, 8.0 * len, st);
    HIPCHK(launch_norm2(v, len, h->partial, h->dnorm, st));
    return STH_OK;
}

static int read_norm(sth_handle* h, const double* v, long len, hipStream_t st, double* out) {
    int rc = norm2_dev(h, v, len, st);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(h->hnorm, h->dnorm, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *out = std::sqrt(h->hnorm[0]);
    return STH_OK;
}

// ---------------------------------------------------------------------------
// Iteration in the spatial eigenbasis.  The multigrid iterates are kept as
// u^ with u = (I (x) U_x) u^; every operator of the cycle (L_h, D^{-1},
// P_t (x) I, its transpose) maps to a pointwise operator over the spatial
// modes, so the cycle runs without spatial transforms.  The transforms are
// applied to f once (f^ = (I (x) U_x^T) f), to the residual once per cycle
// for the stopping test (r = (I (x) C_x) r^, C = M_1 U = U^{-T}), and to the
// result (u = (I (x) U_x) u^).  In exact arithmetic the iterates are those of
// the nodal cycle.
// ---------------------------------------------------------------------------
enum SpatialKind { FWD_U, INV_U, FWD_C, INV_C };

// out = (A^T (x) ... (x) A^T) in (FWD) or (A (x) ... (x) A) in (INV) on every
// time row of `rows` rows; A = U or C.  prec (sth_prec) is the arithmetic of
// the transforms; epi 1 (inverse only) adds the result to out instead of
// storing it; io_f32 2 (forward) writes out as float, 1 (inverse) reads in
// as float (FP32 eigenbasis vectors).  in, out and tmp (a level-0 sized
// scratch vector, used by the axis-by-axis path) must be distinct; the 3-D
// inverse with epi 1 and the 3-D transforms with float data also need a
// second scratch vector tmp2 (which may be `in` for a forward transform).
static int spatial_apply(sth_handle* h, SpatialKind kind, const double* in, double* out, long rows, double* tmp,
                         hipStream_t st, const int* guard = nullptr, int prec = STH_FP64, int epi = 0,
                         double* tmp2 = nullptr, int io_f32 = 0) {
    const bool fwd = (kind == FWD_U || kind == FWD_C);
    const double* A = (kind == FWD_U || kind == INV_U) ? h->Tf : h->Cf;     // A padded
    const double* At = (kind == FWD_U || kind == INV_U) ? h->Ti : h->Ci;    // A^T padded
    const long n = h->n;
    double dof = (double)rows * h->Nx;
    h->tlev = 0;
    if (epi != 0 && fwd) return fail(STH_EINVAL, "accumulating forward transform");
    if (io_f32 && io_f32 != (fwd ? 2 : 1)) return fail(STH_EINVAL, "float data on the wrong side of a transform");
    if (h->dim == 2 && xform2d_supported(h->np)) {
        Timed tm(h, STH_K_XFORM_2D, 4.0 * n * dof, (epi ? 24.0 : 16.0) * dof, st);
        // eigenbasis rows are eig_modes long: the forward transform writes,
        // and the inverse reads, images at that stride
        const long ld = h->Nxe;
        if (prec == STH_BF16X3)
            // out = M (In M^T) with M = A^T (forward) or A (inverse)
            HIPCHK(launch_xform2d_bf16x3(epi, in, out, fwd ? At : A, h->n, h->np, rows, 1.0, st, guard,
                                         fwd ? 0 : ld, fwd ? ld : 0, io_f32));
        else
            HIPCHK(launch_xform2d(prec, fwd ? 0 : 1, epi, in, out, A, h->n, h->np, rows, 1.0, st, guard,
                                  fwd ? 0 : ld, fwd ? ld : 0, io_f32));
        return STH_OK;
    }
    // axis by axis, ping-ponging between the buffers; with accumulation (or
    // float input) the inverse takes the contiguous axis last, so that its
    // epilogue adds into out; float data go through the strided axis only
    const double* T = fwd ? A : At;
    const int* g = guard;
    int rc;
    if (h->dim == 2) {
        // float eigenbasis data with reduced-precision transforms: the
        // intermediate between the two axes is float as well
        const bool fmid = io_f32 != 0 && prec != STH_FP64;
        if (fwd || (epi == 0 && io_f32 == 0)) {
            if ((rc = xform_x(h, prec, 0, in, tmp, T, rows * n, 1.0, st, g, fmid ? 2 : 0))) return rc;
            if ((rc = xform_s(h, prec, tmp, out, T, rows, n, st, g, fmid ? 3 : io_f32))) return rc;
        } else {
            if ((rc = xform_s(h, prec, in, tmp, T, rows, n, st, g, fmid ? 3 : io_f32))) return rc;
            if ((rc = xform_x(h, prec, epi, tmp, out, T, rows * n, 1.0, st, g, fmid ? 1 : 0))) return rc;
        }
    } else if (epi == 0 && io_f32 == 0) {
        if ((rc = xform_x(h, prec, 0, in, out, T, rows * n * n, 1.0, st, g))) return rc;   // x
        if ((rc = xform_s(h, prec, out, tmp, T, rows * n, n, st, g))) return rc;            // y
        if ((rc = xform_s(h, prec, tmp, out, T, rows, n * n, st, g))) return rc;            // z
    } else if (fwd) {
        if (!tmp2) return fail(STH_EINVAL, "3-D transform into float data without a second scratch vector");
        if ((rc = xform_x(h, prec, 0, in, tmp, T, rows * n * n, 1.0, st, g))) return rc;   // x
        if ((rc = xform_s(h, prec, tmp, tmp2, T, rows * n, n, st, g))) return rc;           // y
        if ((rc = xform_s(h, prec, tmp2, out, T, rows, n * n, st, g, io_f32))) return rc;   // z, float out
    } else {
        if (!tmp2) return fail(STH_EINVAL, "3-D inverse transform without a second scratch vector");
        if ((rc = xform_s(h, prec, in, tmp, T, rows, n * n, st, g, io_f32))) return rc;     // z
        if ((rc = xform_s(h, prec, tmp, tmp2, T, rows * n, n, st, g))) return rc;           // y
        if ((rc = xform_x(h, prec, epi, tmp2, out, T, rows * n * n, 1.0, st, g))) return rc;   // x
    }
    return STH_OK;
}

static double* eig_u(sth_handle* h, int lvl, int which) {
    if (lvl == 0) return which == 0 ? h->e1 : (which == 1 ? h->e2 : h->e3);
    if (h->f32) return which ? h->eu2[lvl] : h->eu[lvl];
    return which ? h->lu2[lvl] : h->lu[lvl];
}
static double* eig_f(sth_handle* h, int lvl) {
    if (lvl == 0) return h->e0;
    return h->f32 ? h->ef[lvl] : h->lf[lvl];
}

static const double* level_ktmt(sth_handle* h, int lvl) { return h->dktmt + (size_t)lvl * 2 * kNt * kNt; }

// one smoothing step on level lvl; ec (not null): add the prolonged coarse
// correction of level lvl+1 first
static int eig_smooth(sth_handle* h, int lvl, bool zero_guess, hipStream_t st, const double* ec = nullptr) {
    h->tlev = lvl;
    long S = h->lev_S[lvl];
    double dof = (double)S * slab_len(h);
    int c = h->ecur[lvl];
    double bytes = (zero_guess ? 16.0 : 24.0) * dof + (ec ? 4.0 * dof : 0.0);
    Timed tm(h, STH_K_EIG_SMOOTH, dof * (8.0 * h->Nt + 8.0 + (ec ? 2.0 * h->Nt : 0.0)), bytes, st);
    HIPCHK(launch_eig_smooth(h->dim, h->Nt, h->mixes[lvl], level_ktmt(h, lvl), h->mu1, h->n, eig_f(h, lvl),
                             eig_u(h, lvl, c), eig_u(h, lvl, 1 - c), S, h->omega, zero_guess, ec, h->tr, st,
                             h->guard));
    h->ecur[lvl] = 1 - c;
    return STH_OK;
}

// slabs per thread in the chained passes: the longest chain (fewest repeated
// chain starts) that still leaves min_threads threads; chains of 16 and 32
// slabs only where four times as many threads remain (large levels, where
// the repeated starts of shorter chains cost a measurable share of the
// traffic)
static int chain_length(const sth_handle* h, long S, long min_threads) {
    for (int c : {32, 16})
        if (S % c == 0 && (S / c) * h->Nx >= 4 * min_threads) return c;
    for (int c : {8, 4})
        if (S % c == 0 && (S / c) * h->Nx >= min_threads) return c;
    return 2;
}

static int eig_vcycle(sth_handle* h, int lvl, bool zero_guess, hipStream_t st) {
    h->tlev = lvl;
    if (lvl > 0) h->ecur[lvl] = 0;
    long S = h->lev_S[lvl];
    if (lvl == h->L - 1) {
        double dof = (double)S * slab_len(h);
        Timed tm(h, STH_K_TIMEMIX, dof * (4.0 * h->Nt + 4.0), 16.0 * dof, st);
        HIPCHK(launch_timemix(h->dim, h->Nt, h->mixes[lvl], h->mu1, h->n, h->Nxe, eig_f(h, lvl),
                              eig_u(h, lvl, h->ecur[lvl]), S, true, st, h->guard, h->f32));
        return STH_OK;
    }
    int rc;
    if (lvl == h->L - 3 && lvl > 0 && zero_guess && h->fuse_tail3) {
        // descent over two levels, exact coarsest solve and post-smoothing of
        // the last three levels from this level's right-hand side in one pass
        double dof = (double)S * slab_len(h);
        Timed tm(h, STH_K_EIG_COARSE, dof * (12.0 * h->Nt + 14.0), 16.0 * dof, st);
        HIPCHK(launch_eig_coarse_tail3(h->dim, h->Nt, h->dmix + lvl, h->dmix + lvl + 1, h->dmix + lvl + 2,
                                       h->mixes[lvl].schur != 0, h->mu1, h->n, eig_f(h, lvl), eig_u(h, lvl, 0),
                                       h->tr, h->omega, S, st, h->guard, h->f32));
        h->ecur[lvl] = 0;
        return STH_OK;
    }
    if (lvl == h->L - 2 && lvl > 0 && zero_guess && h->fuse_tail) {
        // descent, exact coarsest solve and post-smoothing of the last two
        // levels from this level's right-hand side in one pass
        double dof = (double)S * slab_len(h);
        Timed tm(h, STH_K_EIG_COARSE, dof * (10.0 * h->Nt + 11.0), 16.0 * dof, st);
        HIPCHK(launch_eig_coarse_tail(h->dim, h->Nt, h->dmix + lvl, h->dmix + lvl + 1, h->mixes[lvl].schur != 0,
                                      h->mu1, h->n, eig_f(h, lvl), eig_u(h, lvl, 0), h->tr,
                                      h->omega, S, st, h->guard, h->f32));
        h->ecur[lvl] = 0;
        return STH_OK;
    }
    if (zero_guess && h->nu_pre == 0) {
        HIPCHK(launch_fill(eig_u(h, lvl, h->ecur[lvl]), S * eslab_len(h), 0.0, st));
        zero_guess = false;
    }
    bool from_zero = false;             // the pre-smoothing step started from zero (A u = omega f)
    if (lvl == 0 && h->presmoothed) {
        // the cycle-end pass of the previous cycle (or of the initial
        // residual) took the pre-smoothing step and restricted its residual;
        // the previous cycle's result, if unformed, is not needed any more
        h->ecur[0] = h->pre_idx;
        h->presmoothed = false;
        h->unformed = sth_handle::Unformed{};
    } else if (zero_guess && h->nu_pre == 1) {
        // one pass: smoothing step from zero and restriction of its residual
        from_zero = true;
        double dof = (double)S * slab_len(h);
        const int c = h->ecur[lvl];
        Timed tm(h, STH_K_EIG_SMOOTH, dof * (8.0 * h->Nt + 8.0), 20.0 * dof, st);
        HIPCHK(launch_eig_down(h->dim, h->Nt, h->mixes[lvl], level_ktmt(h, lvl), h->mu1, h->n, eig_f(h, lvl),
                               eig_u(h, lvl, 1 - c), eig_f(h, lvl + 1), h->tr, h->omega, S, chain_length(h, S, 262144), st,
                               h->guard, h->f32));
        h->ecur[lvl] = 1 - c;
    } else {
        for (int i = 0; i < h->nu_pre; ++i)
            if ((rc = eig_smooth(h, lvl, zero_guess && i == 0, st))) return rc;
        h->tlev = lvl;
        long Sc = h->lev_S[lvl + 1];
        double dof = (double)S * slab_len(h);
        Timed tm(h, STH_K_EIG_RESID, dof * (4.0 * h->Nt + 2.0 * h->Nt), dof * 16.0 + 0.5 * dof * 8.0, st);
        HIPCHK(launch_eig_resid_restrict(h->dim, h->Nt, h->tr, level_ktmt(h, lvl), h->mu1, h->n, eig_f(h, lvl),
                                         eig_u(h, lvl, h->ecur[lvl]), eig_f(h, lvl + 1), Sc, st));
    }
    if ((rc = eig_vcycle(h, lvl + 1, true, st))) return rc;
    h->tlev = lvl;
    const double* ec = eig_u(h, lvl + 1, h->ecur[lvl + 1]);
    if (lvl == 0 && h->defer_close) {
        // prolongation and post-smoothing go into the fused cycle close
        h->pending_ec = ec;
        return STH_OK;
    }
    if (h->nu_post == 0) return prolong_lvl(h, lvl, ec, eig_u(h, lvl, h->ecur[lvl]), st, h->Nxe);
    int first = 0;
    if (from_zero) {
        // the first post-smoothing step in closed form (A u = omega f):
        // reads u and the coarse correction only
        double dof = (double)S * slab_len(h);
        const int c = h->ecur[lvl];
        Timed tm(h, STH_K_EIG_SMOOTH, dof * (4.0 * h->Nt + 4.0), 20.0 * dof, st);
        HIPCHK(launch_eig_post(h->dim, h->Nt, h->mixes[lvl], h->mu1, h->n, eig_u(h, lvl, c), ec, eig_u(h, lvl, 1 - c),
                               h->tr, h->omega, S, chain_length(h, S, 262144), st, h->guard, h->f32));
        h->ecur[lvl] = 1 - c;
        first = 1;
    }
    for (int i = first; i < h->nu_post; ++i)
        if ((rc = eig_smooth(h, lvl, false, st, i == 0 ? ec : nullptr))) return rc;
    return STH_OK;
}

// ||r^||^2 of the residual r^ = f^ - L u^ of the current eigenbasis iterate
// to the pinned host scalars of a norm slot (not synchronised).  With one
// pre-smoothing step in the cycle and a level below, a single pass (the
// cycle-end kernel) also takes the next cycle's smoothing step (into the
// other buffer of the pair) and restricts the residual of its result into
// the next level's right-hand side; the next V-cycle adopts both.

static int eig_residual_cheap(sth_handle* h, hipStream_t st) {
    h->tlev = 0;
    const long S = h->lev_S[0];
    const long len = S * eslab_len(h);             // eigenbasis layout (padded rows)
    const double dof = (double)S * slab_len(h);
    const int c = h->ecur[0];
    if (h->pending_ec) {
        // the cycle's prolongation and post-smoothing step, the residual norm
        // of its result, the next pre-smoothing step and its restriction:
        // the pre-smoothed iterate is read from buffer c, the result goes to
        // the buffer that is neither c nor the next pre-smoothed one, so
        // consecutive cycles alternate between two buffer states
        const double Nt = h->Nt;
        const int cur = c == 0 ? 1 : 0, nxt = 3 - c - cur;
        // norm slot of this cycle: by its next pre-smoothed buffer, so that
        // consecutive cycles alternate (the guard of the next cycle reads it)
        const int slot = nxt == 2 ? 1 : 0;
        CycleFlag flag;
        if (h->guard) flag = CycleFlag{h->dgo + slot, h->hflag_dev + slot, h->dthr, h->nb_lo};
        if (flag.dev && h->poll_seq) {
            flag.seq = h->hseq_dev + slot;
            flag.seq_val = h->last_seq = ++h->seq_counter;
        }
        const int chain = chain_length(h, S, 65536);
        // in the solve loop the result is formed only if it is read
        const bool lazy = h->lazy_close;
        {
            // the pass alone (its final sums are a launch of their own)
            Timed tm(h, STH_K_EIG_CYCLE_CLOSE, dof * (12.0 * Nt + 24.0), (lazy ? 32.0 : 40.0) * dof, st);
            HIPCHK(launch_eig_cycle_close(h->dim, h->Nt, h->mixes[0], level_ktmt(h, 0), h->mu1, h->n, h->e0,
                                          eig_u(h, 0, c), h->pending_ec, lazy ? nullptr : eig_u(h, 0, cur),
                                          eig_u(h, 0, nxt), eig_f(h, 1), h->tr, h->omega, S, chain, h->vw,
                                          h->cpartial, h->n_cpartial, h->dnorm + slot_base(slot),
                                          h->hnorm_dev + slot_base(slot), st, h->guard, flag, false, h->f32));
        }
        h->unformed = lazy ? sth_handle::Unformed{true, c, cur, h->pending_ec} : sth_handle::Unformed{};
        HIPCHK(launch_cycle_sums(h->dim, h->n, S, chain, h->cpartial, h->dnorm + slot_base(slot),
                                 h->hnorm_dev + slot_base(slot), st, h->guard, flag));
        h->last_slot = slot;
        h->pending_ec = nullptr;
        h->wsum_valid = true;
        h->ecur[0] = cur;
        h->pre_idx = nxt;
        h->presmoothed = true;
        return STH_OK;
    }
    if (h->nu_pre == 1 && h->L > 1) {
        const double Nt = h->Nt;
        const int o = c == 0 ? 1 : 0;   // buffer of the pre-smoothed iterate
        Timed tm(h, STH_K_EIG_CYCLE_END, dof * (12.0 * Nt + 10.0), 28.0 * dof, st);
        // with the first cycles enqueued behind it, the initial pass keeps its
        // sums and flag apart from the two alternating cycle slots (the
        // second cycle writes slot 0 while the host reads these)
        CycleFlag flag;
        if (h->first_flag) flag = CycleFlag{h->dgo + 3, h->hflag_dev + 3, h->dthr, h->nb_lo};
        const int at = slot_base(h->first_flag ? 2 : 0);
        // the zero guess of a solve's start is read through its device flag
        const int* unz = (h->unformed.on && h->unformed.zero && h->unformed.dst == c) ? h->zero_in : nullptr;
        HIPCHK(launch_eig_cycle_end(h->dim, h->Nt, h->mixes[0], level_ktmt(h, 0), h->mu1, h->n, h->e0,
                                    eig_u(h, 0, c), eig_u(h, 0, o), eig_f(h, 1), h->tr, h->omega, S,
                                    chain_length(h, S, 65536), h->vw, h->cpartial, h->n_cpartial, h->dnorm + at,
                                    h->hnorm_dev + at, st, flag, h->f32, unz));
        h->wsum_valid = true;
        h->last_slot = 0;
        h->pre_idx = o;
        h->presmoothed = true;
        return STH_OK;                  // the pass stored its sums to the host itself
    }
    {
        Timed tm(h, STH_K_EIG_RESID, dof * 4.0 * h->Nt, dof * 24.0, st);
        HIPCHK(launch_eig_residual(h->dim, h->Nt, level_ktmt(h, 0), h->mu1, h->n, h->e0, eig_u(h, 0, c),
                                   h->buf0, S, st));
    }
    {
        Timed tm(h, STH_K_NORM, 2.0 * dof, 8.0 * dof, st);
        HIPCHK(launch_norm2(h->buf0, len, h->partial, h->dnorm + slot_base(0), st));
    }
    h->wsum_valid = false;
    h->last_slot = 0;
    HIPCHK(hipMemcpyAsync(h->hnorm + slot_base(0), h->dnorm + slot_base(0), sizeof(double), hipMemcpyDeviceToHost,
                          st));
    return STH_OK;
}

// The result of the last cycle when its close left it unformed: the
// post-smoothing step of that close again, from the same inputs, stored
// alone (bitwise the value the close would have stored).
static int form_result(sth_handle* h, hipStream_t st) {
    if (!h->unformed.on) return STH_OK;
    const sth_handle::Unformed uf = h->unformed;
    h->unformed = sth_handle::Unformed{};
    if (uf.dst != h->ecur[0]) return fail(STH_EINVAL, "unformed result in a buffer that is not the iterate");
    h->tlev = 0;
    const long S = h->lev_S[0];
    const double dof = (double)S * slab_len(h);
    if (uf.zero) {
        HIPCHK(launch_fill(eig_u(h, 0, uf.dst), S * eslab_len(h), 0.0, st, uf.zguard, h->f32));
        return STH_OK;
    }
    Timed tm(h, STH_K_EIG_SMOOTH, dof * (10.0 * h->Nt + 8.0), 28.0 * dof, st);
    HIPCHK(launch_eig_cycle_close(h->dim, h->Nt, h->mixes[0], level_ktmt(h, 0), h->mu1, h->n, h->e0,
                                  eig_u(h, 0, uf.c), uf.ec, eig_u(h, 0, uf.dst), nullptr, nullptr, h->tr, h->omega,
                                  S, chain_length(h, S, 65536), h->vw, nullptr, 0, nullptr, nullptr, st, nullptr,
                                  CycleFlag{}, false, h->f32));
    return STH_OK;
}

// The B-spline residual norm ||(I (x) C_x) r^||^2 (C = M_1 U = U^{-T}) of
// the current eigenbasis iterate to hnorm[0] (not synchronised); r^ is
// formed again in buf0.
static int eig_exact_norm(sth_handle* h, hipStream_t st, const CycleFlag& fin = CycleFlag{}) {
    int rc = form_result(h, st);
    if (rc) return rc;
    h->tlev = 0;
    const long S = h->lev_S[0];
    const long len = S * eslab_len(h);             // eigenbasis layout (padded rows)
    const double dof = (double)S * slab_len(h);
    const long rows = S * h->Nt;
    {
        Timed tm(h, STH_K_EIG_RESID, dof * 4.0 * h->Nt, dof * 24.0, st);
        HIPCHK(launch_eig_residual(h->dim, h->Nt, level_ktmt(h, 0), h->mu1, h->n, h->e0, eig_u(h, 0, h->ecur[0]),
                                   h->buf0, S, st));
    }
    if (h->dim == 2 && xform2d_supported(h->np)) {
        // ||C r^ C^T||^2 per image as <r^ G, G r^> (G = C^T C), r not formed
        Timed tm(h, STH_K_RESNORM, dof * 4.0 * h->n, dof * 8.0, st);
        HIPCHK(launch_gram_norm2d(h->buf0, h->Gf, h->n, h->np, rows, h->partial, kNormBlocks, h->dnorm,
                                  h->hnorm_dev, st, fin, h->Nxe));
        return STH_OK;                  // stored hnorm[0] itself
    }
    if (h->dim == 2) {
        // per-axis transforms buf0 -> buf1 -> buf0
        if ((rc = spatial_apply(h, INV_C, h->buf0, h->buf0, rows, h->buf1, st))) return rc;
        if ((rc = norm2_dev(h, h->buf0, len, st))) return rc;
    } else {
        // x: buf0 -> buf1, y: buf1 -> buf0, z: buf0 -> buf1
        if ((rc = spatial_apply(h, INV_C, h->buf0, h->buf1, rows, h->buf0, st))) return rc;
        if ((rc = norm2_dev(h, h->buf1, len, st))) return rc;
    }
    HIPCHK(hipMemcpyAsync(h->hnorm, h->dnorm, sizeof(double), hipMemcpyDeviceToHost, st));
    return STH_OK;
}

// ---------------------------------------------------------------------------
// Device scratch of the entry point that allocates nothing
// (sth_load_rhs_noalloc): the staging of the mode tables of the load vector
// lives in a file-scope device array instead of memory allocated per call.
// Each GPU holds its own copy of the array at its own address, taken once per
// device with that device current; host code passes that address, never the
// array's name, to kernels and copies.
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = size_t(1) << 19;          // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

// device address of the current device's copy of `scratch`
static int scratch_address(double** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(STH_EINVAL, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(STH_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return STH_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
static Problem to_problem(const sth_problem* p) {
    Problem q;
    q.dim = p->dim;
    q.n_elem = p->n_elem;
    q.degree = p->degree;
    q.n_slabs = p->n_slabs;
    q.n_elem_t = p->n_elem_t;
    q.T = p->T;
    q.theta = p->theta;
    q.omega = p->omega;
    q.nu_pre = p->nu_pre;
    q.nu_post = p->nu_post;
    q.prec = p->transform_prec;
    q.coarse_slabs = p->coarse_slabs;
    q.basis = p->iterate_basis;
    q.temporal = p->temporal_form;
    q.space_ratio = p->space_ratio;
    q.minres_iters = p->minres_iters;
    return q;
}

extern "C" {

void sth_problem_default(sth_problem* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->T = 1.0;
    p->theta = 0.01;
    p->omega = 0.5;
    p->nu_pre = 1;
    p->nu_post = 1;
    p->transform_prec = STH_FP64;
    p->coarse_slabs = 128;           // exact parallel-in-time solve; with the level above: one pass
    p->iterate_basis = 0;
    p->temporal_form = 2;
}

const char* sth_last_error(void) { return g_err.c_str(); }

static size_t level_count(const Problem& q) {
    size_t L = 1;
    long S = q.n_slabs;
    while (S > q.coarse_slabs && S % 2 == 0 && (q.level_cap <= 0 || (int)L < q.level_cap)) { S /= 2; ++L; }
    return L;
}

// The post-smoothing step of the finest level goes into the cycle-end pass
// (one more iterate buffer) for V(1,1) cycles in the eigenbasis with a level
// below and N_t <= 5 (the register budget of the fused pass).
static bool fused_cycle_close(const Problem& q, size_t levels) {
    return q.basis == 1 && q.nu_pre == 1 && q.nu_post == 1 && levels > 1 && q.Nt() <= 5;
}

// Eigenbasis vectors in FP32 (arithmetic in FP64): the mixed precision form
// (eigenbasis iteration, reduced-precision transforms) with the fused V(1,1)
// passes and a transform path that reads and writes float data
static bool f32_storage(const Problem& q, size_t levels) {
    const int n = q.n(), np = (n + 15) / 16 * 16;
    return q.basis == 1 && q.prec != STH_FP64 && fused_cycle_close(q, levels) &&
           ((q.dim == 2 && xform2d_supported(np)) || xform_panel_f32_io(np));
}

static size_t workspace_of(Problem q);

int sth_workspace_bytes(const sth_problem* p, size_t* bytes) {
    if (!p || !bytes) return fail(STH_EINVAL, "null argument");
    Problem q = to_problem(p);
    std::string e = validate(q);
    if (!e.empty()) return fail(STH_EINVAL, e);
    *bytes = workspace_of(q);
    return STH_OK;
}

}  // extern "C"

// device bytes of the setup of q and of the problems below it on coarser
// spatial meshes (the same allocations as setup_problem)
static size_t workspace_of(Problem q) {
    const int own = space_transition(q);
    if (own > 0) q.level_cap = own;
    long n = q.n(), np = (n + 15) / 16 * 16;
    long Nx = n * n * (q.dim == 3 ? n : 1);
    if (q.basis == 1) Nx = std::max(Nx, eig_modes(q.dim, (int)n));   // eigenbasis rows are padded
    long slab = (long)q.Nt() * Nx;
    size_t total = 0;
    total += 2 * sizeof(double) * np * np;                   // transforms
    total += sizeof(double) * n * (1 + 2 * (2 * q.degree + 1));
    const bool f32 = f32_storage(q, level_count(q));
    const size_t evecs0 = q.basis == 1 ? 3 + (fused_cycle_close(q, level_count(q)) ? 1 : 0) : 0;   // f^, u^ (x2 or 3)
    total += 2 * sizeof(double) * (size_t)q.n_slabs * slab;                            // buf0, buf1
    total += evecs0 * (f32 ? sizeof(float) : sizeof(double)) * (size_t)q.n_slabs * slab;
    // per coarse level: u, f (nodal), and the eigenbasis u^, its partner and
    // f^ (the u, f pair shared unless the eigenbasis vectors are float)
    const size_t vecsl_bytes = 2 * sizeof(double) + (q.basis == 1 ? (f32 ? 3 * sizeof(float) : sizeof(double)) : 0);
    if (q.basis == 1) {
        total += 3 * sizeof(double) * np * np;                // C, C^T, G
        total += sizeof(double) * (2 * (((size_t)(q.n_slabs / 2) * (size_t)(Nx) + 255) / 256) + 1);   // cycle-end partials
        total += sizeof(double) * 2 * n;                                 // mode weights
    }
    long S = q.n_slabs;
    size_t L = level_count(q);
    for (size_t l = 1; l < L; ++l) {
        S /= 2;
        total += vecsl_bytes * (size_t)S * slab;
    }
    total += sizeof(double) * (kNormBlocks + kNormSlots + L * 2 * kNt * kNt) + sizeof(TimeMix) * L;
    if (q.minres_iters > 0)   // eight MinRes vectors of the finest level and the per-system scalars
        total += sizeof(double) * (size_t)q.n_slabs * slab * 8 + sizeof(double) * q.n_slabs * (kNt / 2) * kMrState;
    if (own > 0) {
        // the coarse-mesh problem, its finest right-hand side and iterate,
        // and the band tables of P_x
        Problem c = q;
        c.n_elem = q.n_elem / 2;
        c.n_slabs = (int)(S / 2);
        c.theta = q.theta * ((double)c.n_slabs / q.n_slabs);
        c.level_cap = 0;
        total += workspace_of(c);
        const long nc = c.n();
        total += 2 * sizeof(double) * (size_t)c.n_slabs * q.Nt() * nc * nc * (q.dim == 3 ? nc : 1);
        total += (size_t)(n + nc) * (sizeof(int) + sizeof(double) * (q.degree + 2));
    }
    return total;
}

extern "C" {

size_t sth_problem_vector_len(const sth_problem* p) {
    if (!p) return 0;
    Problem q = to_problem(p);
    if (!validate(q).empty()) return 0;
    long n = q.n();
    return (size_t)q.n_slabs * q.Nt() * n * n * (q.dim == 3 ? n : 1);
}

}  // extern "C"

static int setup_problem(Problem q, hipStream_t s, sth_handle** out);

extern "C" {

int sth_setup(const sth_problem* p, void* stream, sth_handle** out) {
    if (!p || !out) return fail(STH_EINVAL, "null argument");
    *out = nullptr;
    Problem q = to_problem(p);
    std::string e = validate(q);
    if (!e.empty()) return fail(STH_EINVAL, e);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STH_ENODEV, "no HIP device");
    {
        // the scratch address of this device, taken once at set-up
        double* scr = nullptr;
        const int rc = scratch_address(&scr);
        if (rc != STH_OK) return rc;
    }
    return setup_problem(q, (hipStream_t)stream, out);
}

}  // extern "C"

// The problem on the halved spatial mesh below the last level of h (a
// space-time coarsening step): n_elem / 2 elements per axis, half the slabs
// of that level on the same (0, T), and theta scaled by a power of two so
// that sigma is the finest one (the Galerkin coarse operators are the
// rediscretisations with the finest sigma), then P_x as two band tables.
static int attach_coarse_space(sth_handle* h, const Problem& q, hipStream_t s) {
    Problem c = q;
    c.n_elem = q.n_elem / 2;
    c.n_slabs = (int)(h->lev_S[h->L - 1] / 2);
    c.theta = q.theta * ((double)c.n_slabs / q.n_slabs);
    c.level_cap = 0;
    int rc = setup_problem(c, s, &h->child);
    if (rc) return rc;
    const int nf = h->n, nc = h->child->n;
    h->n_c = nc;
    Mat Px;
    space_prolongation(c.n_elem, q.degree, Px);
    if (Px.r != nf || Px.c != nc) return fail(STH_EINVAL, "spatial prolongation has the wrong shape");
    // band of output o: the inputs with a nonzero coefficient, shifted to
    // stay inside [0, n_in) at the common width W (zeros fill the rest)
    auto band = [&](bool restr, std::vector<int>& j0, std::vector<double>& co, int& W) {
        const int nout = restr ? nc : nf, nin = restr ? nf : nc;
        auto at = [&](int o, int i) { return restr ? Px(i, o) : Px(o, i); };
        std::vector<int> lo(nout, nin), hi(nout, -1);
        for (int o = 0; o < nout; ++o)
            for (int i = 0; i < nin; ++i)
                if (at(o, i) != 0.0) {
                    lo[o] = std::min(lo[o], i);
                    hi[o] = std::max(hi[o], i);
                }
        W = 1;
        for (int o = 0; o < nout; ++o)
            if (hi[o] >= lo[o]) W = std::max(W, hi[o] - lo[o] + 1);
        j0.assign(nout, 0);
        co.assign((size_t)nout * W, 0.0);
        for (int o = 0; o < nout; ++o) {
            const int a = std::max(0, std::min(hi[o] >= lo[o] ? lo[o] : 0, nin - W));
            j0[o] = a;
            for (int k = 0; k < W; ++k) co[(size_t)o * W + k] = at(o, a + k);
        }
    };
    std::vector<int> rj0, pj0;
    std::vector<double> rco, pco;
    band(true, rj0, rco, h->rW);
    band(false, pj0, pco, h->pW);
    const size_t clen = (size_t)h->child->lev_S[0] * slab_len(h->child);
    if (hipMalloc((void**)&h->rj0, sizeof(int) * rj0.size()) != hipSuccess ||
        hipMalloc((void**)&h->pj0, sizeof(int) * pj0.size()) != hipSuccess ||
        hipMalloc((void**)&h->rco, sizeof(double) * rco.size()) != hipSuccess ||
        hipMalloc((void**)&h->pco, sizeof(double) * pco.size()) != hipSuccess ||
        hipMalloc((void**)&h->cf, sizeof(double) * clen) != hipSuccess ||
        hipMalloc((void**)&h->cu, sizeof(double) * clen) != hipSuccess)
        return fail(STH_ENOMEM, "device allocation failed");
    if (hipMemcpyAsync(h->rj0, rj0.data(), sizeof(int) * rj0.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->pj0, pj0.data(), sizeof(int) * pj0.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->rco, rco.data(), sizeof(double) * rco.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->pco, pco.data(), sizeof(double) * pco.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(STH_EHIP, "upload of the spatial prolongation failed");
    return STH_OK;
}

static int setup_problem(Problem q, hipStream_t s, sth_handle** out) {
    *out = nullptr;
    // levels on this spatial mesh (all of them unless the hierarchy
    // coarsens in space below one of them)
    const int own = space_transition(q);
    if (own > 0) q.level_cap = own;
    std::string e;
    sth_handle* h = new sth_handle();
    int st = build_setup(q, h->S, e);
    if (st != 0) {
        delete h;
        return fail(st, e);
    }
    h->dim = q.dim;
    h->n = h->S.n;
    h->np = (h->n + 15) / 16 * 16;
    h->split = h->S.half > 0 && h->np == h->n && xform_split_supported(h->n);
    h->Nt = h->S.Nt;
    h->p = q.degree;
    h->Nx = (long)h->n * h->n * (q.dim == 3 ? h->n : 1);
    h->Nxe = eig_modes(q.dim, h->n);
    h->omega = q.omega;
    h->nu_pre = q.nu_pre;
    h->nu_post = q.nu_post;
    h->prec = q.prec;
    h->basis = q.basis;
    if (h->basis != 0 && h->basis != 1) {
        delete h;
        return fail(STH_EINVAL, "iterate_basis must be 0 or 1");
    }
    h->L = (int)h->S.levels.size();
    h->nb_lo = std::pow(h->S.m1_min, h->dim);
    h->nb_hi = std::pow(h->S.m1_max, h->dim);
    h->fuse_close = fused_cycle_close(q, (size_t)h->L);
    h->f32 = f32_storage(q, (size_t)h->L);
    {
        int G = 0, LA = 0;
        h->fuse_tail = h->basis == 1 && h->nu_pre == 1 && h->nu_post == 1 && h->L >= 3 &&
                       h->S.levels[h->L - 2].schur == h->S.levels[h->L - 1].schur &&
                       coarse_tail_shape(h->Nt, h->S.levels[h->L - 2].S, &G, &LA);
        h->fuse_tail3 = h->basis == 1 && h->nu_pre == 1 && h->nu_post == 1 && h->L >= 4 &&
                        h->S.levels[h->L - 3].schur == h->S.levels[h->L - 1].schur &&
                        h->S.levels[h->L - 2].schur == h->S.levels[h->L - 1].schur &&
                        coarse_tail3_shape(h->Nt, h->S.levels[h->L - 3].S, &G, &LA);
    }
    for (auto& lv : h->S.levels) {
        h->lev_S.push_back(lv.S);
        TimeOp op{};
        TimeMix tm{};
        // eigen form: complex pairs first, so that each occupies an aligned
        // 2x2 block, then the real eigenvalues (slot k holds column perm[k])
        std::vector<int> perm;
        if (!lv.schur) {
            for (int i = 0; i < h->Nt; ++i)
                if (lv.kind[i] == 1) { perm.push_back(i); perm.push_back(i + 1); }
            for (int i = 0; i < h->Nt; ++i)
                if (lv.kind[i] == 0) perm.push_back(i);
        } else {
            for (int i = 0; i < h->Nt; ++i) perm.push_back(i);
        }
        if ((int)perm.size() != h->Nt) {
            delete h;
            return fail(STH_ECOND, "temporal eigen form: unpaired complex eigenvalue");
        }
        for (int i = 0; i < h->Nt; ++i) {
            const int pi = perm[i];
            for (int j = 0; j < h->Nt; ++j) {
                op.Kt[i * kNt + j] = lv.Kt(i, j);
                op.Mt[i * kNt + j] = lv.Mt(i, j);
                tm.W[i * kNt + j] = lv.W(pi, j);
                tm.V[i * kNt + j] = lv.V(i, perm[j]);
            }
            if (lv.schur) {
                tm.kind[i] = lv.kind[i];
                for (int j = 0; j < h->Nt; ++j) tm.R[i * kNt + j] = lv.R(i, j);
            } else {
                tm.zd[i] = lv.re[pi];
                tm.zo[i] = lv.kind[pi] == 0 ? 0.0 : lv.im[pi];
            }
        }
        tm.schur = lv.schur ? 1 : 0;
        h->ops.push_back(op);
        h->mixes.push_back(tm);
    }
    if (h->L > 1 || own > 0) {
        // P_t of every time step of this handle, also of a space-time step
        // below its last level (the map does not depend on the slab length)
        Mat P;
        time_prolongation(q.n_elem_t, q.degree, P);
        for (int i = 0; i < 2 * h->Nt; ++i)
            for (int j = 0; j < h->Nt; ++j) h->tr.P[i * kNt + j] = P(i, j);
    }
    // host staging of the spatial factors
    int n = h->n, np = h->np, B = 2 * h->p + 1;
    std::vector<double> Tf((size_t)np * np, 0.0), Ti((size_t)np * np, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            Tf[(size_t)i * np + j] = h->S.U(i, j);     // r^_j = sum_i U_ij r_i
            Ti[(size_t)j * np + i] = h->S.U(i, j);     // z_i  = sum_j U_ij z^_j
        }
    std::vector<double> M1b((size_t)n * B, 0.0), K1b((size_t)n * B, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < B; ++k) {
            int j = i - h->p + k;
            if (j >= 0 && j < n) {
                M1b[(size_t)i * B + k] = h->S.M1(i, j);
                K1b[(size_t)i * B + k] = h->S.K1(i, j);
            }
        }
    auto cleanup = [&](int code, const std::string& msg) {
        sth_destroy(h);
        return fail(code, msg);
    };
    auto dalloc = [&](double** ptr, size_t count) -> bool {
        return hipMalloc((void**)ptr, std::max<size_t>(count, 1) * sizeof(double)) == hipSuccess;
    };
    // buffers both iterations use hold either layout
    const long slab = h->basis == 1 ? std::max(slab_len(h), eslab_len(h)) : slab_len(h);
    const long eslab = eslab_len(h);
    if (!dalloc(&h->Tf, (size_t)np * np) || !dalloc(&h->Ti, (size_t)np * np) || !dalloc(&h->mu1, n) ||
        !dalloc(&h->M1b, (size_t)n * B) || !dalloc(&h->K1b, (size_t)n * B) ||
        !dalloc(&h->buf0, (size_t)q.n_slabs * slab) || !dalloc(&h->buf1, (size_t)q.n_slabs * slab) ||
        !dalloc(&h->partial, kNormBlocks) || !dalloc(&h->dnorm, kNormSlots) ||
        !dalloc(&h->dktmt, (size_t)h->L * 2 * kNt * kNt))
        return cleanup(STH_ENOMEM, "device allocation failed");
    std::vector<double> ktmt((size_t)h->L * 2 * kNt * kNt);
    for (int l = 0; l < h->L; ++l) {
        std::memcpy(&ktmt[(size_t)l * 2 * kNt * kNt], h->ops[l].Kt, sizeof(double) * kNt * kNt);
        std::memcpy(&ktmt[(size_t)l * 2 * kNt * kNt + kNt * kNt], h->ops[l].Mt, sizeof(double) * kNt * kNt);
    }
    h->lu.assign(h->L, nullptr);
    h->lf.assign(h->L, nullptr);
    h->lu2.assign(h->L, nullptr);
    h->ecur.assign(h->L, 0);
    // doubles that hold `count` eigenbasis values (floats with FP32 storage)
    auto ecount = [&](size_t count) { return h->f32 ? (count + 1) / 2 : count; };
    const size_t ebytes = h->f32 ? sizeof(float) : sizeof(double);
    h->eu.assign(h->L, nullptr);
    h->ef.assign(h->L, nullptr);
    h->eu2.assign(h->L, nullptr);
    for (int l = 1; l < h->L; ++l) {
        if (!dalloc(&h->lu[l], (size_t)h->lev_S[l] * slab) || !dalloc(&h->lf[l], (size_t)h->lev_S[l] * slab))
            return cleanup(STH_ENOMEM, "device allocation failed");
        if (h->basis == 1 && !h->f32 && !dalloc(&h->lu2[l], (size_t)h->lev_S[l] * slab))
            return cleanup(STH_ENOMEM, "device allocation failed");
        if (h->f32) {
            const size_t c = ecount((size_t)h->lev_S[l] * slab);
            if (!dalloc(&h->eu[l], c) || !dalloc(&h->ef[l], c) || !dalloc(&h->eu2[l], c))
                return cleanup(STH_ENOMEM, "device allocation failed");
        }
    }
    if (hipMalloc((void**)&h->dmix, sizeof(TimeMix) * h->mixes.size()) != hipSuccess)
        return cleanup(STH_ENOMEM, "device allocation failed");
    if (hipMemcpyAsync(h->dmix, h->mixes.data(), sizeof(TimeMix) * h->mixes.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return cleanup(STH_EHIP, "upload of the setup failed");
    std::vector<double> Cf, Ci, Gf;
    if (h->basis == 1) {
        // C = M_1 U = U^{-T} (from U^T M_1 U = I)
        Cf.assign((size_t)np * np, 0.0);
        Ci.assign((size_t)np * np, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double c = 0.0;
                for (int k = std::max(0, i - h->p); k <= std::min(n - 1, i + h->p); ++k) c += h->S.M1(i, k) * h->S.U(k, j);
                Cf[(size_t)i * np + j] = c;
                Ci[(size_t)j * np + i] = c;
            }
        h->n_cpartial = 3 * (((q.n_slabs / 2) * h->Nxe + 255) / 256);   // three sums per block
        if (!dalloc(&h->cpartial, (size_t)h->n_cpartial) ||
            !dalloc(&h->Cf, (size_t)np * np) || !dalloc(&h->Ci, (size_t)np * np) ||
            !dalloc(&h->e0, ecount((size_t)q.n_slabs * eslab)) || !dalloc(&h->e1, ecount((size_t)q.n_slabs * eslab)) ||
            !dalloc(&h->e2, ecount((size_t)q.n_slabs * eslab)) ||
            (h->fuse_close && !dalloc(&h->e3, ecount((size_t)q.n_slabs * eslab))))
            return cleanup(STH_ENOMEM, "device allocation failed");
        // the padded modes of the eigenbasis vectors start (and stay) zero
        for (double* v : {h->e0, h->e1, h->e2, h->e3})
            if (v && hipMemsetAsync(v, 0, ebytes * (size_t)q.n_slabs * eslab, s) != hipSuccess)
                return cleanup(STH_EHIP, "clearing the eigenbasis vectors failed");
        for (int l = 1; l < h->L; ++l) {
            for (double* v : {h->lu[l], h->lf[l], h->lu2[l]})
                if (v && hipMemsetAsync(v, 0, sizeof(double) * (size_t)h->lev_S[l] * slab, s) != hipSuccess)
                    return cleanup(STH_EHIP, "clearing the eigenbasis vectors failed");
            for (double* v : {h->eu[l], h->ef[l], h->eu2[l]})
                if (v && hipMemsetAsync(v, 0, ebytes * (size_t)h->lev_S[l] * slab, s) != hipSuccess)
                    return cleanup(STH_EHIP, "clearing the eigenbasis vectors failed");
        }
        // mode weights of the lower bound of the B-spline residual norm
        const std::vector<double> vwh = residual_mode_weights(h->S);
        if (!dalloc(&h->vw, (size_t)2 * n))
            return cleanup(STH_ENOMEM, "device allocation failed");
        if (hipMemcpyAsync(h->Cf, Cf.data(), Cf.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(h->Ci, Ci.data(), Ci.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(h->vw, vwh.data(), vwh.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
            return cleanup(STH_EHIP, "upload of the setup failed");
        if (h->dim == 2 && xform2d_supported(np)) {
            // G = C^T C for the exact residual norm
            Gf.assign((size_t)np * np, 0.0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double g = 0.0;
                    for (int k = 0; k < n; ++k) g += Cf[(size_t)k * np + i] * Cf[(size_t)k * np + j];
                    Gf[(size_t)i * np + j] = g;
                }
            if (!dalloc(&h->Gf, (size_t)np * np) ||
                hipMemcpyAsync(h->Gf, Gf.data(), Gf.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
                return cleanup(STH_EHIP, "upload of the setup failed");
        }
    }
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void**)&h->hnorm, kNormSlots * sizeof(double), mapped) != hipSuccess ||
        hipHostMalloc((void**)&h->hflag, 5 * sizeof(int), mapped) != hipSuccess ||
        hipHostMalloc((void**)&h->hseq, 2 * sizeof(int), mapped) != hipSuccess)
        return cleanup(STH_ENOMEM, "pinned host allocation failed");
    h->hseq[0] = h->hseq[1] = 0;
    if (hipHostGetDevicePointer((void**)&h->hnorm_dev, h->hnorm, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&h->hflag_dev, h->hflag, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&h->hseq_dev, h->hseq, 0) != hipSuccess)
        return cleanup(STH_EHIP, "pinned host memory is not mapped");
    if (hipMalloc((void**)&h->dgo, 6 * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&h->dthr, 2 * sizeof(double)) != hipSuccess)
        return cleanup(STH_ENOMEM, "device allocation failed");
    // dgo[5] stays 0: the flag of an inner solve's zero guess
    if (hipMemsetAsync(h->dgo, 0, 6 * sizeof(int), s) != hipSuccess)
        return cleanup(STH_EHIP, "clearing the device flags failed");
    for (auto& e : h->evring)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return cleanup(STH_EHIP, "event creation failed");
    if (hipMemcpyAsync(h->Tf, Tf.data(), Tf.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->Ti, Ti.data(), Ti.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->mu1, h->S.mu.data(), (size_t)n * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->M1b, M1b.data(), M1b.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->K1b, K1b.data(), K1b.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->dktmt, ktmt.data(), ktmt.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(STH_EHIP, "upload of the setup failed");
    if (q.minres_iters > 0) {
        // the temporal blocks of every level: pairs (alpha, beta_1, beta_2)
        // in the leading 2x2 blocks, real eigenvalues after them
        h->minres = q.minres_iters;
        int max_pairs = 0;
        for (int l = 0; l < h->L; ++l) {
            const TimeMix& tm = h->mixes[l];
            if (tm.schur)
                return cleanup(STH_EINVAL, "the MinRes slab inverse needs the temporal eigen form on every level "
                                           "(the automatic form chose the real Schur form)");
            PairOps ops{};
            TimeRowMix win{}, vout{};
            PinvRows pr{};
            int np = 0;
            while (2 * np + 1 < h->Nt && tm.zo[2 * np] != 0.0) ++np;
            for (int k = np; 2 * k + 1 < h->Nt; ++k)
                if (tm.zo[2 * k] != 0.0 || tm.zo[2 * k + 1] != 0.0)
                    return cleanup(STH_EINVAL, "temporal eigen form: complex pairs are not the leading blocks");
            ops.npairs = np;
            for (int t = 0; t < h->Nt; ++t) {
                win.sin[t] = 1.0;
                win.sout[t] = 1.0;
                vout.sin[t] = 1.0;
                vout.sout[t] = 1.0;
                pr.scale[t] = 1.0;
                pr.shift[t] = tm.zd[t];              // a real eigenvalue: K_x + lambda M_x
                for (int j = 0; j < h->Nt; ++j) {
                    win.M[t * kNt + j] = tm.W[t * kNt + j];
                    vout.M[t * kNt + j] = tm.V[t * kNt + j];
                }
            }
            for (int k = 0; k < np; ++k) {
                const double a = tm.zd[2 * k], b1 = tm.zo[2 * k], b2 = tm.zo[2 * k + 1];
                const double s = std::sqrt(std::fabs(b1 * b2));
                ops.alpha[k] = a;
                ops.a11[k] = std::fabs(b2);
                ops.a12[k] = -b1 * std::fabs(b2);
                ops.a21[k] = std::fabs(b1) * b2;
                ops.a22[k] = -std::fabs(b1);
                win.sout[2 * k] = std::fabs(b2);
                win.sout[2 * k + 1] = std::fabs(b1);
                pr.scale[2 * k] = 1.0 / std::fabs(b2);
                pr.scale[2 * k + 1] = 1.0 / std::fabs(b1);
                pr.shift[2 * k] = pr.shift[2 * k + 1] = a + s;
                vout.sin[2 * k + 1] = -1.0;
            }
            h->mr_ops.push_back(ops);
            h->mr_win.push_back(win);
            h->mr_vout.push_back(vout);
            h->mr_pinv.push_back(pr);
            max_pairs = std::max(max_pairs, np);
        }
        const size_t vlen = (size_t)h->lev_S[0] * slab_len(h);
        for (double*& v : h->mr)
            if (!dalloc(&v, vlen)) return cleanup(STH_ENOMEM, "device allocation failed");
        if (!dalloc(&h->mrst, (size_t)h->lev_S[0] * std::max(max_pairs, 1) * kMrState))
            return cleanup(STH_ENOMEM, "device allocation failed");
    }
    if (own > 0) {
        if ((h->L != own)) return cleanup(STH_EINVAL, "level count of the spatial mesh");
        const int rc = attach_coarse_space(h, q, s);
        if (rc) {
            const std::string msg = g_err;
            return cleanup(rc, msg);
        }
    }
    *out = h;
    return STH_OK;
}

extern "C" {

size_t sth_vector_len(const sth_handle* h) { return h ? (size_t)h->lev_S[0] * slab_len(h) : 0; }

}  // extern "C"

// The handle of the chain (h, its child, ...) that holds multigrid level
// `level`, with `level` made local to it; null past the coarsest level.
static sth_handle* level_owner(const sth_handle* h, int& level) {
    sth_handle* o = const_cast<sth_handle*>(h);
    if (level < 0) return nullptr;
    while (o && level >= o->L) {
        level -= o->L;
        o = o->child;
    }
    return o;
}

extern "C" {

size_t sth_level_len(const sth_handle* h, int level) {
    const sth_handle* o = level_owner(h, level);
    if (!o) return 0;
    return (size_t)o->lev_S[level] * slab_len(o);
}

int sth_num_levels(const sth_handle* h) {
    int L = 0;
    for (; h; h = h->child) L += h->L;
    return L;
}

int sth_level_elems(const sth_handle* h, int level) {
    const sth_handle* o = level_owner(h, level);
    return o ? o->S.prob.n_elem : 0;
}

int sth_load_rhs(sth_handle* h, const sth_rhs_modes* m, double* f, void* stream) {
    if (!h || !m || !f) return fail(STH_EINVAL, "null argument");
    if (m->n_modes < 0 || (m->n_modes > 0 && (!m->amp || !m->k || !m->omega || !m->phase)))
        return fail(STH_EINVAL, "bad mode list");
    hipStream_t st = (hipStream_t)stream;
    const Problem& q = h->S.prob;
    long S = q.n_slabs;
    int n = h->n, Nt = h->Nt, M = m->n_modes;
    if (M == 0) {
        HIPCHK(launch_fill(f, S * slab_len(h), 0.0, st));
        return STH_OK;
    }
    std::vector<double> T((size_t)M * S * Nt), X((size_t)M * 3 * n, 0.0), tmp;
    for (int q2 = 0; q2 < M; ++q2) {
        load_time(q, m->omega[q2], m->phase[q2], tmp);
        for (size_t i = 0; i < tmp.size(); ++i) T[(size_t)q2 * S * Nt + i] = m->amp[q2] * tmp[i];
        for (int a = 0; a < h->dim; ++a) {
            load_space(q, m->k[q2 * h->dim + a], tmp);
            for (int i = 0; i < n; ++i) X[(size_t)q2 * 3 * n + (size_t)a * n + i] = tmp[i];
        }
    }
    double *dT = nullptr, *dX = nullptr;
    if (hipMalloc((void**)&dT, T.size() * 8) != hipSuccess) return fail(STH_ENOMEM, "rhs staging");
    if (hipMalloc((void**)&dX, X.size() * 8) != hipSuccess) {
        (void)hipFree(dT);
        return fail(STH_ENOMEM, "rhs staging");
    }
    hipError_t e1 = hipMemcpyAsync(dT, T.data(), T.size() * 8, hipMemcpyHostToDevice, st);
    hipError_t e2 = hipMemcpyAsync(dX, X.data(), X.size() * 8, hipMemcpyHostToDevice, st);
    hipError_t e3 = launch_rhs(h->dim, Nt, n, M, dT, dX, f, S, st);
    hipError_t e4 = hipStreamSynchronize(st);
    (void)hipFree(dT);
    (void)hipFree(dX);
    if (e1 || e2 || e3 || e4) return fail(STH_EHIP, "rhs assembly failed");
    return STH_OK;
}

int sth_load_rhs_noalloc(sth_handle* h, const sth_rhs_modes* m, double* f, void* stream) {
    if (!h || !m || !f) return fail(STH_EINVAL, "null argument");
    if (m->n_modes < 0 || (m->n_modes > 0 && (!m->amp || !m->k || !m->omega || !m->phase)))
        return fail(STH_EINVAL, "bad mode list");
    hipStream_t st = (hipStream_t)stream;
    const Problem& q = h->S.prob;
    const long S = q.n_slabs;
    const int n = h->n, Nt = h->Nt, M = m->n_modes;
    if (M == 0) {
        HIPCHK(launch_fill(f, S * slab_len(h), 0.0, st));
        return STH_OK;
    }
    // the temporal and spatial tables side by side in the scratch array
    const size_t nT = (size_t)M * S * Nt, nX = (size_t)M * 3 * n;
    if (nT + nX > kScratchDoubles)
        return fail(STH_EINVAL, "mode tables of " + std::to_string(nT + nX) + " doubles exceed the scratch of " +
                                    std::to_string(kScratchDoubles) + " doubles (4 MiB): fewer modes or slabs");
    double* scr = nullptr;
    int rc = scratch_address(&scr);
    if (rc != STH_OK) return rc;
    std::vector<double> T(nT), X(nX, 0.0), tmp;
    for (int q2 = 0; q2 < M; ++q2) {
        load_time(q, m->omega[q2], m->phase[q2], tmp);
        for (size_t i = 0; i < tmp.size(); ++i) T[(size_t)q2 * S * Nt + i] = m->amp[q2] * tmp[i];
        for (int a = 0; a < h->dim; ++a) {
            load_space(q, m->k[q2 * h->dim + a], tmp);
            for (int i = 0; i < n; ++i) X[(size_t)q2 * 3 * n + (size_t)a * n + i] = tmp[i];
        }
    }
    HIPCHK(hipMemcpyAsync(scr, T.data(), nT * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(scr + nT, X.data(), nX * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(launch_rhs(h->dim, Nt, n, M, scr, scr + nT, f, S, st));
    HIPCHK(hipStreamSynchronize(st));     // the host tables go out of scope
    return STH_OK;
}

int sth_apply(sth_handle* h, const double* u, double* y, void* stream) {
    if (!h || !u || !y) return fail(STH_EINVAL, "null argument");
    return residual(h, 0, nullptr, u, y, 0, h->lev_S[0], -1.0, (hipStream_t)stream);
}

int sth_residual(sth_handle* h, const double* f, const double* u, double* r, void* stream) {
    if (!h || !f || !u || !r) return fail(STH_EINVAL, "null argument");
    return residual(h, 0, f, u, r, 0, h->lev_S[0], 1.0, (hipStream_t)stream);
}

int sth_block_solve(sth_handle* h, const double* r, double* z, void* stream) {
    if (!h || !r || !z) return fail(STH_EINVAL, "null argument");
    if (r == h->buf0 || z == h->buf0) return fail(STH_EINVAL, "aliasing");
    if (h->minres) return minres_slab_inverse(h, 0, r, z, 2, 1.0, h->lev_S[0], (hipStream_t)stream);
    return slab_inverse(h, 0, r, z, 2, 1.0, 0, h->lev_S[0], (hipStream_t)stream);
}

int sth_smooth(sth_handle* h, const double* f, double* u, int steps, void* stream) {
    if (!h || !f || !u || steps < 0) return fail(STH_EINVAL, "bad argument");
    for (int i = 0; i < steps; ++i) {
        int rc = smooth_step(h, 0, f, u, false, (hipStream_t)stream);
        if (rc) return rc;
    }
    return STH_OK;
}

int sth_vcycle(sth_handle* h, const double* f, double* u, void* stream) {
    if (!h || !f || !u) return fail(STH_EINVAL, "null argument");
    return vcycle_lvl(h, 0, f, u, false, (hipStream_t)stream);
}

// one solve iteration: V-cycle, residual into buf1, its squared norm copied
// to the pinned host scalar (not synchronised)
static int solve_iteration(sth_handle* h, const double* f, double* u, hipStream_t st) {
    int rc;
    long len = h->lev_S[0] * slab_len(h);
    if (h->basis == 1) {
        h->defer_close = h->fuse_close;
        // a speculative solve guards every launch of the cycle with the
        // continuation flag of the cycle before it (its norm slot)
        h->guard = h->sv.spec && h->presmoothed ? h->dgo + (h->pre_idx == 2 ? 1 : 0) : nullptr;
        if (h->guard && h->first_guard) h->guard = h->dgo + 3;   // the initial pass's flag
        h->first_guard = false;
        rc = eig_vcycle(h, 0, false, st);
        h->defer_close = false;
        h->lazy_close = true;
        if (rc == STH_OK) rc = eig_residual_cheap(h, st);
        h->lazy_close = false;
        h->pending_ec = nullptr;
        h->guard = nullptr;
        return rc;
    }
    if ((rc = vcycle_lvl(h, 0, f, u, false, st))) return rc;
    if ((rc = residual(h, 0, f, u, h->buf1, 0, h->lev_S[0], 1.0, st))) return rc;
    if ((rc = norm2_dev(h, h->buf1, len, st))) return rc;
    HIPCHK(hipMemcpyAsync(h->hnorm, h->dnorm, sizeof(double), hipMemcpyDeviceToHost, st));
    return STH_OK;
}

// Captures solve_iteration into a HIP graph for (f, u); replays are cheaper
// to launch than the individual kernels and may go to any stream.  Not used
// on the legacy default stream, where capture is not allowed.  Enqueues one
// iteration without waiting for it.
static int graph_launch(sth_handle* h, const double* f, double* u, hipStream_t st) {
    // level-0 buffer state at entry (eigenbasis): iterate, pre-smoothed iterate
    const int key = h->basis == 1 ? h->ecur[0] + 3 * h->pre_idx + 9 * (h->presmoothed ? 1 : 0) +
                                        18 * (h->sv.spec ? 1 : 0)
                                  : 0;
    const unsigned mask = h->timing ? h->timing_mask : 0u;
    sth_handle::GraphEntry* g = nullptr;
    for (auto& e : h->gent)
        if (e.exec && e.f == f && e.u == u && e.key == key && e.mask == mask) g = &e;
    if (!g) {
        if (!h->allow_capture) {                          // capture later; run this one eagerly
            h->graph_launched = false;
            return solve_iteration(h, f, u, st);
        }
        // an empty entry, else the least recently used one
        g = &h->gent[0];
        for (auto& e : h->gent) {
            if (!e.exec) { g = &e; break; }
            if (e.last_used < g->last_used) g = &e;
        }
        drop_graph_entry(*g);
        h->grecs.clear();
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        h->capturing = true;
        int rc = solve_iteration(h, f, u, st);
        h->capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            h->grecs.clear();
            return rc;
        }
        HIPCHK(e);
        g->graph = graph;
        HIPCHK(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
        g->f = f;
        g->u = u;
        g->mask = mask;
        g->key = key;
        g->recs.swap(h->grecs);
        g->ecur0_after = h->basis == 1 ? h->ecur[0] : 0;
        g->pre_after = h->pre_idx;
        g->presm_after = h->presmoothed;
        g->slot_after = h->last_slot;
        g->unf_after = h->unformed;
    } else if (h->basis == 1) {
        // a replay does not run the host-side bookkeeping of the capture:
        // take the level-0 buffer state the captured iteration left
        h->ecur[0] = g->ecur0_after;
        h->pre_idx = g->pre_after;
        h->presmoothed = g->presm_after;
        h->last_slot = g->slot_after;
        h->unformed = g->unf_after;
    }
    g->last_used = ++h->graph_clock;
    HIPCHK(hipGraphLaunch(g->exec, st));
    h->glast = g;
    h->graph_launched = true;
    return STH_OK;
}

// after a replay has completed: add the times of its timed launches
static int graph_collect(sth_handle* h) {
    if (!h->glast) return STH_OK;
    for (auto& r : h->glast->recs) {
        float e = 0;
        HIPCHK(hipEventElapsedTime(&e, r.a, r.b));
        h->gms[r.cls] += e;
        h->gfl[r.cls] += r.flops;
        h->gby[r.cls] += r.bytes;
        h->gcnt[r.cls] += 1;
    }
    return STH_OK;
}

}  // extern "C"

namespace sth {

// Asynchronous solve, in three calls that only enqueue work on st; between
// them the caller waits for the stream (sth_solve) or polls an event (the
// serving loop).  solve_begin: ||f||^2 and the initial residual norm^2 to
// the pinned host scalars.
static sth_handle::Snap take_snap(const sth_handle* h);
static int spec_enqueue(sth_handle* h);

// inner (not null): an inner solve of a mixed-precision solve, with ||f|| =
// *inner_fn known on the host and transforms in precision tprec
static int solve_begin_impl(sth_handle* h, const double* f, double* u, double rtol, int maxit, hipStream_t st,
                            const double* inner_fn = nullptr, int tprec = STH_FP64) {
    if (!h || !f || !u || !(rtol >= 0) || maxit < 0) return fail(STH_EINVAL, "bad argument");
    auto& v = h->sv;
    v = sth_handle::SolveState{};
    v.f = f;
    v.u = u;
    v.st = st;
    v.rtol = rtol;
    v.maxit = maxit;
    v.inner = inner_fn != nullptr;
    v.tprec = tprec;
    // cycles enqueued ahead of their predecessor's norm (eigenbasis with the
    // fused cycle close; not while kernels are timed one by one)
    v.spec = h->basis == 1 && h->fuse_close && h->speculate && !h->timing;
    // completion marks instead of per-cycle events: the blocking solve with
    // eager launches (a captured graph would replay fixed marks)
    h->poll_seq = h->want_poll && v.spec && !h->use_graph;
    h->wait_ev = nullptr;
    h->wait_slot = -1;
    h->graph_launched = false;
    h->presmoothed = false;
    h->tlev = 0;
    const long len = h->lev_S[0] * slab_len(h);
    if (v.inner) {
        h->hnorm[1] = (*inner_fn) * (*inner_fn);     // read by the host only
    } else {
        {
            Timed tm(h, STH_K_NORM, 2.0 * len, 8.0 * len, st);
            HIPCHK(launch_norm2(f, len, h->partial, h->dnorm + 1, st));
        }
        HIPCHK(hipMemcpyAsync(h->hnorm + 1, h->dnorm + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    int rc;
    if (h->basis == 1) {
        // f^ = (I (x) U_x^T) f, u^ = (I (x) C_x^T) u (C^T = U^{-1}), then the residual
        const long rows = h->lev_S[0] * h->Nt;
        h->ecur[0] = 0;
        h->unformed = sth_handle::Unformed{};
        // (FP32 eigenbasis vectors: only in inner solves, whose f is the
        // outer residual in buf1 or the caller's f; a 3-D forward transform
        // into float data uses buf1 as its second work vector after its
        // first step has read f)
        if ((rc = spatial_apply(h, FWD_U, f, h->e0, rows, h->buf0, st, nullptr, v.tprec, 0,
                                h->f32 ? h->buf1 : nullptr, h->f32 ? 2 : 0)))
            return rc;
        h->tlev = 0;
        // with the initial pass next (cycle-end kernel), a zero guess is not
        // written: that pass reads the device flag instead, and the buffer is
        // filled only if it is read as the iterate (form_result)
        const bool lazy_zero = h->nu_pre == 1 && h->L > 1;
        const int* zg = nullptr;
        if (v.inner) {
            zg = h->dgo + 5;                            // holds 0: the guess is zero
            if (!lazy_zero) HIPCHK(launch_fill(h->e1, h->lev_S[0] * eslab_len(h), 0.0, st, nullptr, h->f32));
        } else {
            // an initial guess of zeros (the usual start) needs no transform:
            // a device flag says whether u has a nonzero entry; the transform
            // runs only then, the fill of zeros only otherwise
            int* nz = h->dgo + 4;
            zg = nz;
            HIPCHK(launch_any_nonzero(u, len, nz, st));
            if ((rc = spatial_apply(h, FWD_C, u, h->e1, rows, h->buf0, st, nz))) return rc;
            if (!lazy_zero) HIPCHK(launch_fill(h->e1, h->lev_S[0] * eslab_len(h), 0.0, st, nz, h->f32));
        }
        if (lazy_zero) {
            h->unformed = sth_handle::Unformed{};
            h->unformed.on = true;
            h->unformed.zero = true;
            h->unformed.dst = 0;
            h->unformed.zguard = zg;
            h->zero_in = zg;
        }
        // (with graph replay, whose captured cycles have fixed guards, the
        // first cycle waits for the initial norms instead)
        if (!v.spec || maxit < 1 || h->use_graph) return eig_residual_cheap(h, st);
        // speculation from the start: the threshold on the device, the
        // initial pass sets the flag that guards the first cycle, and the
        // first cycles go behind it without waiting for the norms
        if (v.inner) {
            const double t = rtol * (*inner_fn);
            HIPCHK(launch_set_flag(h->dgo + 3, 0, st, h->dthr, t * t, t));
        } else {
            HIPCHK(launch_spec_threshold(h->dthr, h->dnorm + 1, rtol, st));
        }
        h->first_flag = true;
        rc = eig_residual_cheap(h, st);
        h->first_flag = false;
        if (rc) return rc;
        v.s0 = take_snap(h);
        h->first_guard = true;
        if ((rc = spec_enqueue(h))) return rc;
        v.phase = 4;                    // (enqueue_iteration sets phase 1)
        return STH_OK;
    }
    if ((rc = residual(h, 0, f, u, h->buf1, 0, h->lev_S[0], 1.0, st))) return rc;
    if ((rc = norm2_dev(h, h->buf1, len, st))) return rc;
    HIPCHK(hipMemcpyAsync(h->hnorm, h->dnorm, sizeof(double), hipMemcpyDeviceToHost, st));
    return STH_OK;
}

static bool solve_should_stop(const sth_handle::SolveState& v) {
    return !(v.rn > v.rtol * v.fn) || v.it >= v.maxit || !std::isfinite(v.rn) || v.growth >= 3;
}

static int enqueue_iteration(sth_handle* h) {
    auto& v = h->sv;
    v.phase = 1;
    // kernel timing records events around individual launches, so it runs
    // the iterations eagerly
    if (v.st != nullptr && h->use_graph && !h->timing) return graph_launch(h, v.f, v.u, v.st);
    h->graph_launched = false;
    return solve_iteration(h, v.f, v.u, v.st);
}

static hipEvent_t next_event(sth_handle* h) {
    hipEvent_t e = h->evring[h->evnext];
    h->evnext = (h->evnext + 1) % 4;
    return e;
}

static sth_handle::Snap take_snap(const sth_handle* h) {
    return sth_handle::Snap{h->ecur[0], h->pre_idx, h->presmoothed, h->last_slot, h->last_seq, h->unformed};
}

// Completion of the cycle just enqueued: an event, or nothing to record when
// its final sum leaves a completion mark (poll_seq)
static int mark_cycle(sth_handle* h, hipEvent_t* ev) {
    *ev = nullptr;
    if (h->poll_seq) return STH_OK;
    *ev = next_event(h);
    HIPCHK(hipEventRecord(*ev, h->sv.st));
    return STH_OK;
}

// the caller's next wait: for cycle s (its event or its completion mark)
static void wait_for(sth_handle* h, const sth_handle::Snap& s, hipEvent_t ev) {
    h->wait_ev = ev;
    h->wait_slot = h->poll_seq ? s.slot : -1;
    h->wait_seq = s.seqv;
}

static void put_snap(sth_handle* h, const sth_handle::Snap& s) {
    h->ecur[0] = s.ecur0;
    h->pre_idx = s.pre_idx;
    h->presmoothed = s.presmoothed;
    h->last_slot = s.slot;
    h->unformed = s.unf;
}

// Enqueues the next cycle (it must run: the flag it is guarded by holds 1)
// and, while maxit allows, one more behind it guarded by the first one's
// flag.  The caller then waits for the first.
static int spec_enqueue(sth_handle* h) {
    auto& v = h->sv;
    int rc = enqueue_iteration(h);
    if (rc) return rc;
    v.a = take_snap(h);
    if ((rc = mark_cycle(h, &v.ev_a))) return rc;
    v.pend = 0;
    if (v.it + 2 <= v.maxit) {
        if ((rc = enqueue_iteration(h))) return rc;
        v.b = take_snap(h);
        if ((rc = mark_cycle(h, &v.ev_b))) return rc;
        v.pend = 1;
    }
    wait_for(h, v.a, v.ev_a);
    return STH_OK;
}

static int solve_finish(sth_handle* h, bool* more) {
    auto& v = h->sv;
    *more = false;
    v.phase = 2;
    h->wait_ev = nullptr;
    h->wait_slot = -1;
    int rc = form_result(h, v.st);
    if (rc) return rc;
    // u = (I (x) U_x) u^ (an inner solve adds it to u, unless u is zero)
    return spatial_apply(h, INV_U, eig_u(h, 0, h->ecur[0]), v.u, h->lev_S[0] * h->Nt, h->buf0, v.st, nullptr,
                         v.tprec, (v.inner && !v.inner_store) ? 1 : 0, h->buf1, h->f32 ? 1 : 0);
}

// Lower bound of the B-spline residual norm of the cycle whose sums are in
// norm slot `slot` (the larger of the two bounds of solve_continue); slot 2
// holds the initial pass of a speculative solve
static double eig_lower_bound(const sth_handle* h, int slot) {
    const double ssq = h->hnorm[slot_base(slot)], wsq = h->hnorm[slot_base(slot) + 1];
    double lo2 = h->nb_lo * ssq;
    if (h->wsum_valid && std::isfinite(wsq)) lo2 = std::max(lo2, (1.0 - 1e-8) * wsq);
    return std::sqrt(lo2);
}

// Upper bound of the B-spline residual norm of the same cycle: the smaller
// of nb_hi ||r^||^2 (the eigenvalues of G = C^T C are those of M_1) and
// sum_m w_m r^_m^2 with w_m = prod a over the axes of mode m (a the absolute
// row sums of G; the Schur test bounds x^T (G (x) G) x by the absolute row
// sums of G (x) G), slightly enlarged against rounding.  When it meets the
// tolerance the cycle has converged without the exact norm; with the lower
// bound above the tolerance it provably has not, so the cycle count is that
// of the plain stopping test either way.
static double eig_upper_bound(const sth_handle* h, int slot) {
    const double ssq = h->hnorm[slot_base(slot)], usq = h->hnorm[slot_base(slot) + 2];
    double up2 = h->nb_hi * ssq;
    if (h->wsum_valid && std::isfinite(usq)) up2 = std::min(up2, (1.0 + 1e-8) * usq);
    return std::sqrt(up2);
}

// Exact norm of the current iterate in the speculative loop; on the fused
// 2-D path the mapping of the result into u goes right behind it, guarded by
// the device's copy of the host's final test (unguarded when the cycle count
// or growth already ends the solve), so the end of a solve needs no host
// round trip.  A mapping that runs although the solve goes on is overwritten
// by the final one.
static int spec_exact_norm(sth_handle* h) {
    auto& v = h->sv;
    v.phase = 3;
    v.fin_enq = false;
    h->wait_ev = nullptr;
    h->wait_slot = -1;
    if (!(h->dim == 2 && xform2d_supported(h->np))) return eig_exact_norm(h, v.st);
    v.fin_always = v.it >= v.maxit || v.growth >= 3;
    const CycleFlag fin = v.fin_always ? CycleFlag{} : CycleFlag{h->dgo + 2, h->hflag_dev + 2, h->dthr, 0.0, 1};
    int rc = eig_exact_norm(h, v.st, fin);
    if (rc) return rc;
    if ((rc = spatial_apply(h, INV_U, eig_u(h, 0, h->ecur[0]), v.u, h->lev_S[0] * h->Nt, h->buf0, v.st,
                            v.fin_always ? nullptr : h->dgo + 2)))
        return rc;
    v.fin_enq = true;
    return STH_OK;
}

// Speculative form of solve_continue: after cycle k's event, its flag (set
// on the device from the same bound the plain loop tests) says whether cycle
// k+1, already enqueued behind it, runs; if not, cycle k+1 leaves every
// buffer as it was, the host state goes back to cycle k's, and the exact
// norm of cycle k's result decides as in the plain loop.  The cycle count
// and the iterates are those of the plain loop.
static int solve_continue_spec(sth_handle* h, bool* more) {
    auto& v = h->sv;
    const double target = v.rtol * v.fn;
    *more = true;
    if (v.phase == 0) {
        v.fn = std::sqrt(h->hnorm[1]);
        if (v.fn == 0.0) v.fn = 1.0;
        const double r = std::sqrt(h->hnorm[slot_base(0)]);
        v.prev = r;
        v.rn = eig_lower_bound(h, 0);
        if (!std::isfinite(r) || v.maxit == 0) return solve_finish(h, more);
        if (!(v.rn > v.rtol * v.fn)) {
            if (v.inner) return solve_finish(h, more);      // the outer loop takes the exact norm
            const double up = eig_upper_bound(h, 0);
            if (up <= v.rtol * v.fn) {
                v.rn = up;
                return solve_finish(h, more);
            }
            v.phase = 3;
            int rc = eig_exact_norm(h, v.st);
            h->wait_ev = nullptr;
            h->wait_slot = -1;
            return rc;
        }
        // arm the first cycle and set the threshold of the cycles' flags
        HIPCHK(launch_set_flag(h->dgo + h->last_slot, 1, v.st, h->dthr, (v.rtol * v.fn) * (v.rtol * v.fn),
                                  v.rtol * v.fn));
        v.phase = 1;
        return spec_enqueue(h);
    }
    if (v.phase == 4) {
        // the initial norms and cycle a are done; the flag of the initial
        // pass (its own norm slot 2 and flag hflag[3]) says
        // whether cycle a (and so cycle b) ran
        v.fn = std::sqrt(h->hnorm[1]);
        if (v.fn == 0.0) v.fn = 1.0;
        const double r = std::sqrt(h->hnorm[slot_base(2)]);
        v.prev = r;
        v.phase = 1;
        if (h->hflag[3] == 0) {
            put_snap(h, v.s0);
            v.pend = 0;
            v.rn = eig_lower_bound(h, 2);
            if (!std::isfinite(r)) {
                v.rn = r;
                return solve_finish(h, more);
            }
            if (v.inner) return solve_finish(h, more);
            const double up = eig_upper_bound(h, 2);
            if (up <= v.rtol * v.fn) {
                v.rn = up;
                return solve_finish(h, more);
            }
            return spec_exact_norm(h);
        }
        // cycle a ran: go on as after any completed cycle
    }
    if (v.phase == 3) {
        v.rn = std::sqrt(h->hnorm[0]);
        if (!std::isfinite(v.rn) || !(v.rn > target) || v.it >= v.maxit || v.growth >= 3) {
            if (v.fin_enq && (v.fin_always || h->hflag[2] != 0)) {
                // the mapping into u ran behind the norm
                v.phase = 2;
                *more = false;
                return STH_OK;
            }
            return solve_finish(h, more);
        }
        // not converged: the next cycle runs after all
        HIPCHK(launch_set_flag(h->dgo + h->last_slot, 1, v.st, h->dthr, (v.rtol * v.fn) * (v.rtol * v.fn),
                                  v.rtol * v.fn));
        v.phase = 1;
        return spec_enqueue(h);
    }
    // cycle a has completed
    ++v.it;
    const int slot = v.a.slot;
    const double r = std::sqrt(h->hnorm[slot_base(slot)]);
    if (std::isfinite(r)) {
        v.growth = (r > v.prev) ? v.growth + 1 : 0;
        v.prev = r;
    }
    v.rn = eig_lower_bound(h, slot);
    if (v.drain) return solve_finish(h, more);
    const bool go = h->hflag[slot] != 0;
    if (go) {
        if (v.growth >= 3 && v.pend) {
            // cycle b runs: take it as the last one
            v.a = v.b;
            v.ev_a = v.ev_b;
            v.pend = 0;
            v.drain = true;
            wait_for(h, v.a, v.ev_a);
            return STH_OK;
        }
        if (v.growth >= 3 || v.it >= v.maxit) return solve_finish(h, more);
        if (v.pend) {
            // cycle b is real: wait for it, with the next one guarded behind it
            v.a = v.b;
            v.ev_a = v.ev_b;
            v.pend = 0;
            wait_for(h, v.a, v.ev_a);
            if (v.it + 2 <= v.maxit) {
                int rc = enqueue_iteration(h);
                if (rc) return rc;
                v.b = take_snap(h);
                if ((rc = mark_cycle(h, &v.ev_b))) return rc;
                v.pend = 1;
            }
            return STH_OK;
        }
        return spec_enqueue(h);
    }
    // the bound does not exclude convergence (or a sum is not finite):
    // cycle b, if any, leaves everything untouched
    if (v.pend) {
        put_snap(h, v.a);
        v.pend = 0;
    }
    if (!std::isfinite(r)) {
        v.rn = r;
        return solve_finish(h, more);
    }
    if (v.inner) return solve_finish(h, more);
    const double up = eig_upper_bound(h, slot);
    if (up <= target) {
        v.rn = up;
        return solve_finish(h, more);
    }
    return spec_exact_norm(h);
}

// Once the work enqueued by the previous call has completed: read the
// residual norm, then enqueue either the next iteration (*more = true) or
// the final mapping of the result into u (*more = false).
//
// Eigenbasis iteration: every cycle yields ||r^|| of its residual in the
// eigenbasis and a lower bound of the B-spline residual norm: ||r||^2 =
// r^T (I (x) G (x) G) r^ (G = C^T C) is at least nb_lo ||r^||^2 (the
// eigenvalues of G are those of M_1, nb_lo = lambda_min(M_1)^dim) and at
// least sum_m v_m r^_m^2 with v_m = 2 prod d - prod a over the axes (d the
// diagonal of G, a its absolute row sums: G (x) G - D (x) D is bounded by its
// row sums).  The second is within a few per cent of ||r||^2 when G is nearly
// diagonal, as for B-spline mass matrices.  While the bound exceeds
// rtol ||f|| the cycle is provably not converged and the next one starts at
// once; otherwise the exact ||r|| is evaluated and decides, as it would in
// every cycle, so the cycle count is that of the plain stopping test.
// Growth is watched on ||r^||.
static int solve_continue_impl(sth_handle* h, bool* more) {
    auto& v = h->sv;
    *more = false;
    if (v.phase == 2) return STH_OK;
    if (h->graph_launched) {
        int rc = graph_collect(h);
        if (rc) return rc;
        h->graph_launched = false;
    }
    if (v.spec) return solve_continue_spec(h, more);
    const bool eig = h->basis == 1;
    if (v.phase == 3) {
        v.rn = std::sqrt(h->hnorm[0]);
    } else {
        const double r = std::sqrt(h->hnorm[eig ? slot_base(h->last_slot) : 0]);
        if (v.phase == 0) {
            v.fn = std::sqrt(h->hnorm[1]);
            if (v.fn == 0.0) v.fn = 1.0;
            v.prev = r;
        } else {
            ++v.it;
            if (std::isfinite(r)) {
                v.growth = (r > v.prev) ? v.growth + 1 : 0;
                v.prev = r;
            }
        }
        v.rn = r;
        if (eig) {
            // lower bound of ||r||: the larger of nb_lo ||r^||^2 and the
            // mode-weighted sum (slightly reduced against rounding)
            v.rn = eig_lower_bound(h, h->last_slot);
            *more = true;
            if (std::isfinite(r) && v.rn > v.rtol * v.fn && v.it < v.maxit && v.growth < 3)
                return enqueue_iteration(h);
            if (v.inner) return solve_finish(h, more);
            const double up = eig_upper_bound(h, h->last_slot);
            if (std::isfinite(r) && up <= v.rtol * v.fn) {
                v.rn = up;
                return solve_finish(h, more);
            }
            v.phase = 3;
            return eig_exact_norm(h, v.st);
        }
    }
    if (!solve_should_stop(v)) {
        *more = true;
        return enqueue_iteration(h);
    }
    v.phase = 2;
    if (eig) {
        // u = (I (x) U_x) u^
        int rc = form_result(h, v.st);
        if (rc) return rc;
        return spatial_apply(h, INV_U, eig_u(h, 0, h->ecur[0]), v.u, h->lev_S[0] * h->Nt, h->buf0, v.st);
    }
    return STH_OK;
}

// ---------------------------------------------------------------------------
// Mixed precision (eigenbasis iteration, transform_prec FP32 or BF16x3): the
// spatial transforms run in reduced precision, so f^ and the mapping back
// carry their rounding; an FP64 defect correction wins the accuracy back.
// Each outer step forms the B-spline residual r = f - L_h u in FP64 (the
// residual kernel of the nodal iteration) and its exact norm, which is the
// stopping test of Section 4.4; an inner eigenbasis solve then reduces r by a
// factor eta (set by the transform precision, or just what the tolerance
// needs) from a zero guess, and its result is added to u by the
// reduced-precision inverse transform.  An inverse accurate to 1e-4 keeps the
// multigrid's iteration count (Section 4.4), so the inner cycles are those of
// the FP64 solve split over two or three outer steps.
// ---------------------------------------------------------------------------
// Smallest residual reduction asked of an inner solve.  The cycle count of a
// solve hardly depends on how it splits over the outer steps (the inner
// reductions multiply), but every outer step costs a residual pass and four
// transforms: these values let the 2-D problem with 256 x 256 elements and
// 1024 slabs (relative residual 1e-8) finish in two outer steps with 11 (FP32)
// or 13 (BF16x3) cycles, where 1e-6 took 13 cycles and 1e-4 in BF16x3 a third
// outer step.
static double mixed_inner_eta(int prec) { return prec == STH_BF16X3 ? 2e-5 : 3e-5; }

static int mixed_residual(sth_handle* h) {
    auto& m = h->mx;
    const long S = h->lev_S[0];
    const long len = S * slab_len(h);
    h->tlev = 0;
    if (residual_norm_fused(h->dim, h->n, h->p, h->Nt)) {
        // the residual kernel sums the squares of its output itself
        const double dof = (double)len;
        Timed tm(h, STH_K_RESIDUAL, dof * (10.0 * (2 * h->p + 1) + 4.0 * h->Nt + 4.0), dof * 24.0, m.st);
        HIPCHK(launch_residual_norm(h->dim, h->Nt, h->p, h->n, h->M1b, h->K1b, level_ktmt(h, 0), m.f, m.u, h->buf1,
                                    S, h->cpartial, h->n_cpartial, h->dnorm + kMixR, h->hnorm_dev + kMixR, m.st));
    } else {
        int rc = residual(h, 0, m.f, m.u, h->buf1, 0, S, 1.0, m.st);
        if (rc) return rc;
        h->tlev = 0;
        {
            Timed tm(h, STH_K_NORM, 2.0 * len, 8.0 * len, m.st);
            HIPCHK(launch_norm2(h->buf1, len, h->partial, h->dnorm + kMixR, m.st));
        }
        HIPCHK(hipMemcpyAsync(h->hnorm + kMixR, h->dnorm + kMixR, sizeof(double), hipMemcpyDeviceToHost, m.st));
    }
    h->wait_ev = nullptr;                 // the caller waits for the stream
    h->wait_slot = -1;
    m.phase = 0;
    return STH_OK;
}

static int mixed_begin(sth_handle* h, const double* f, double* u, double rtol, int maxit, hipStream_t st) {
    if (!h || !f || !u || !(rtol >= 0) || maxit < 0) return fail(STH_EINVAL, "bad argument");
    auto& m = h->mx;
    m = sth_handle::Mixed{};
    m.on = true;
    m.f = f;
    m.u = u;
    m.st = st;
    m.rtol = rtol;
    m.maxit = maxit;
    h->sv = sth_handle::SolveState{};
    h->sv.st = st;
    h->graph_launched = false;
    h->presmoothed = false;
    const long len = h->lev_S[0] * slab_len(h);
    h->tlev = 0;
    {
        Timed tm(h, STH_K_NORM, 2.0 * len, 8.0 * len, st);
        HIPCHK(launch_norm2(f, len, h->partial, h->dnorm + kMixF, st));
    }
    HIPCHK(hipMemcpyAsync(h->hnorm + kMixF, h->dnorm + kMixF, sizeof(double), hipMemcpyDeviceToHost, st));
    // whether u has a nonzero entry: from zero (the usual start) the first
    // outer residual is f itself, and the first inner solve starts on f
    {
        Timed tm(h, STH_K_OTHER, 0.0, 8.0 * len, st);
        HIPCHK(launch_any_nonzero(u, len, h->dgo + 4, st));
    }
    HIPCHK(hipMemcpyAsync(h->hflag + 4, h->dgo + 4, sizeof(int), hipMemcpyDeviceToHost, st));
    m.phase = 3;
    return STH_OK;
}

// the inner solve of L e = r to eta ||r|| (at least what the tolerance needs,
// with a margin), added into u (stored, when u is zero); r is the outer
// residual (buf1) or f
static int mixed_inner(sth_handle* h, const double* r, double rn, bool u_zero = false) {
    auto& m = h->mx;
    const double eta = std::max(mixed_inner_eta(h->prec), 0.5 * m.rtol * m.fn / rn);
    int rc = solve_begin_impl(h, r, m.u, eta, m.maxit - m.it, m.st, &rn, h->prec);
    if (rc) return rc;
    h->sv.inner_store = u_zero;
    m.phase = 1;
    return STH_OK;
}

static int mixed_continue(sth_handle* h, bool* more) {
    auto& m = h->mx;
    *more = false;
    if (m.phase == 2) return STH_OK;
    if (m.phase == 3) {
        m.fn = std::sqrt(h->hnorm[kMixF]);
        if (m.fn == 0.0) m.fn = 1.0;
        if (h->hflag[4] != 0) {
            // nonzero initial guess: its residual first
            m.phase = 0;
            *more = true;
            return mixed_residual(h);
        }
        const double rn = std::sqrt(h->hnorm[kMixF]);
        m.rn = m.prev = rn;
        if (!std::isfinite(rn) || !(rn > m.rtol * m.fn) || m.maxit < 1) {
            m.phase = 2;
            return STH_OK;
        }
        *more = true;
        return mixed_inner(h, m.f, rn, true);
    }
    if (m.phase == 1) {
        bool inner_more = false;
        int rc = solve_continue_impl(h, &inner_more);
        if (rc || inner_more) {
            *more = inner_more;
            return rc;
        }
        // the inner result is being added to u: the next outer residual
        m.it += h->sv.it;
        ++m.outer;
        *more = true;
        return mixed_residual(h);
    }
    // outer residual norm of the current iterate
    if (m.outer == 0) {
        m.fn = std::sqrt(h->hnorm[kMixF]);
        if (m.fn == 0.0) m.fn = 1.0;
    }
    const double rn = std::sqrt(h->hnorm[kMixR]);
    if (m.outer > 0 && std::isfinite(rn)) m.growth = (rn >= m.prev) ? m.growth + 1 : 0;
    m.rn = rn;
    m.prev = rn;
    if (!std::isfinite(rn) || !(rn > m.rtol * m.fn) || m.it >= m.maxit || m.growth >= 3) {
        m.phase = 2;
        return STH_OK;
    }
    *more = true;
    return mixed_inner(h, h->buf1, rn);
}

static int mixed_result(sth_handle* h, int* iters, double* relres) {
    const auto& m = h->mx;
    if (iters) *iters = m.it;
    if (relres) *relres = m.rn / m.fn;
    if (!std::isfinite(m.rn)) return fail(STH_ENOCONV, "residual is not finite");
    if (m.growth >= 3) return fail(STH_ENOCONV, "residual did not decrease over 3 consecutive outer steps");
    if (m.rn > m.rtol * m.fn) return fail(STH_ENOCONV, "maxit reached");
    return STH_OK;
}

// whether sth_solve on this handle takes the mixed-precision route
static bool mixed_route(const sth_handle* h) { return h->basis == 1 && h->prec != STH_FP64; }

int solve_begin(sth_handle* h, const double* f, double* u, double rtol, int maxit, hipStream_t st) {
    if (h) h->mx.on = false;
    if (h && mixed_route(h)) return mixed_begin(h, f, u, rtol, maxit, st);
    return solve_begin_impl(h, f, u, rtol, maxit, st);
}

int solve_continue(sth_handle* h, bool* more) {
    if (h->mx.on) return mixed_continue(h, more);
    return solve_continue_impl(h, more);
}

// Outcome of a finished solve: STH_OK when the tolerance was met.
int solve_result(sth_handle* h, int* iters, double* relres) {
    if (h->mx.on) return mixed_result(h, iters, relres);
    const auto& v = h->sv;
    if (iters) *iters = v.it;
    if (relres) *relres = v.rn / v.fn;
    if (!std::isfinite(v.rn)) return fail(STH_ENOCONV, "residual is not finite");
    if (v.growth >= 3) return fail(STH_ENOCONV, "residual grew over 3 consecutive cycles");
    if (v.rn > v.rtol * v.fn) return fail(STH_ENOCONV, "maxit reached");
    return STH_OK;
}

void solve_allow_capture(sth_handle* h, bool allow) { h->allow_capture = allow; }

hipEvent_t solve_wait_event(sth_handle* h) { return h->wait_ev; }

}  // namespace sth

extern "C" {

// Waits until the final sum of the awaited cycle has left its completion
// mark in mapped memory (it stores the mark after its norms and flag, behind
// a system-scope fence).  After each millisecond of waiting it checks the
// stream, so that a failed launch or a missing mark ends the wait with an
// error; the check is rare because a stream query can itself put work
// between the kernels.
static int wait_mark(sth_handle* h, hipStream_t st) {
    volatile int* p = h->hseq + h->wait_slot;
    const int want = h->wait_seq;
    auto last = std::chrono::steady_clock::now();
    for (long spin = 1; *p != want; ++spin) {
        if ((spin & 1023) != 0) continue;
        const auto now = std::chrono::steady_clock::now();
        if (now - last >= std::chrono::milliseconds(1)) {
            last = now;
            const hipError_t q = hipStreamQuery(st);
            if (q == hipSuccess) {
                if (*p == want) break;
                return fail(STH_EHIP, "cycle completion mark not set");
            }
            if (q != hipErrorNotReady) return fail(STH_EHIP, std::string("stream work failed: ") + hipGetErrorString(q));
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return STH_OK;
}

int sth_solve(sth_handle* h, const double* f, double* u, double rtol, int maxit, int* iters, double* relres,
              void* stream) {
    if (!h || !f || !u || !(rtol >= 0) || maxit < 0) return fail(STH_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    // completion marks instead of per-cycle events (also for the inner
    // solves of a mixed-precision solve, which start inside the loop)
    h->want_poll = true;
    int rc = solve_begin(h, f, u, rtol, maxit, st);
    bool more = true;
    while (rc == STH_OK && more) {
        if (h->wait_slot >= 0) rc = wait_mark(h, st);
        else if (h->wait_ev) HIPCHK(hipEventSynchronize(h->wait_ev));
        else HIPCHK(hipStreamSynchronize(st));
        if (rc == STH_OK) rc = solve_continue(h, &more);
    }
    h->want_poll = false;
    h->poll_seq = false;
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(st));
    return solve_result(h, iters, relres);
}

// ---------------------------------------------------------------------------
// FGMRES(m) outer loop, right-preconditioned by one V-cycle from a zero
// initial guess (the use of the multigrid as a preconditioner named in the
// introduction of the paper).  Flexible: the preconditioned vectors are kept,
// so the preconditioner may change between iterations.  Classical
// Gram-Schmidt applied twice, Givens rotations on the host.
// ---------------------------------------------------------------------------
static int precondition(sth_handle* h, const double* v, double* z, hipStream_t st) {
    if (h->basis == 0) return vcycle_lvl(h, 0, v, z, true, st);
    // the same cycle in the spatial eigenbasis: z = (I (x) U) V((I (x) U^T) v)
    const long rows = h->lev_S[0] * h->Nt;
    int rc;
    // (transforms in the handle's precision: FGMRES is flexible, so a
    // reduced-precision preconditioner leaves its residual test exact)
    if ((rc = spatial_apply(h, FWD_U, v, h->e0, rows, h->buf0, st, nullptr, h->prec, 0, h->buf1, h->f32 ? 2 : 0)))
        return rc;
    h->ecur[0] = 0;
    h->presmoothed = false;
    h->unformed = sth_handle::Unformed{};
    if ((rc = eig_vcycle(h, 0, true, st))) return rc;
    return spatial_apply(h, INV_U, eig_u(h, 0, h->ecur[0]), z, rows, h->buf0, st, nullptr, h->prec, 0, h->buf1,
                         h->f32 ? 1 : 0);
}

static int krylov_workspace(sth_handle* h, int m) {
    if (h->k_alloc >= m) return STH_OK;
    for (double** q : {&h->kv, &h->kz, &h->kc, &h->kpart})
        if (*q) { (void)hipFree(*q); *q = nullptr; }
    if (h->khost) { (void)hipHostFree(h->khost); h->khost = nullptr; }
    h->k_alloc = 0;
    const size_t len = (size_t)h->lev_S[0] * slab_len(h);
    if (hipMalloc((void**)&h->kv, sizeof(double) * len * (m + 1)) != hipSuccess ||
        hipMalloc((void**)&h->kz, sizeof(double) * len * m) != hipSuccess ||
        hipMalloc((void**)&h->kc, sizeof(double) * kMaxKrylov) != hipSuccess ||
        hipMalloc((void**)&h->kpart, sizeof(double) * 1024 * kMaxKrylov) != hipSuccess ||
        hipHostMalloc((void**)&h->khost, sizeof(double) * kMaxKrylov, 0) != hipSuccess)
        return fail(STH_ENOMEM, "FGMRES workspace allocation failed");
    h->k_alloc = m;
    return STH_OK;
}

int sth_solve_fgmres(sth_handle* h, const double* f, double* u, double rtol, int maxit, int restart, int* iters,
                     double* relres, void* stream) {
    if (!h || !f || !u || !(rtol >= 0) || maxit < 0 || restart < 1 || restart >= kMaxKrylov)
        return fail(STH_EINVAL, "bad argument (restart must be in 1..31)");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = krylov_workspace(h, restart))) return rc;
    const long len = h->lev_S[0] * slab_len(h);
    double* V = h->kv;
    double* Z = h->kz;
    double fn = 0.0;
    if ((rc = read_norm(h, f, len, st, &fn))) return rc;
    if (fn == 0.0) fn = 1.0;
    const int m = restart;
    std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), y(m);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    int it = 0;
    double rn = 0.0;
    for (;;) {
        // r = f - L u into V_0, beta = ||r||
        if ((rc = residual(h, 0, f, u, V, 0, h->lev_S[0], 1.0, st))) return rc;
        double beta = 0.0;
        if ((rc = read_norm(h, V, len, st, &beta))) return rc;
        rn = beta;
        if (!std::isfinite(beta)) break;
        if (beta <= rtol * fn || it >= maxit) break;
        h->khost[0] = 1.0 / beta;
        HIPCHK(hipMemcpyAsync(h->kc, h->khost, sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(launch_multiaxpy(V, len, 0, h->kc, 1.0 / beta, V, len, st));       // V_0 = r / beta
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jn = 0;                          // columns completed in this cycle
        for (int j = 0; j < m && it < maxit; ++j) {
            double* Vj = V + (size_t)j * len;
            double* Zj = Z + (size_t)j * len;
            double* w = V + (size_t)(j + 1) * len;
            if ((rc = precondition(h, Vj, Zj, st))) return rc;
            if ((rc = residual(h, 0, nullptr, Zj, w, 0, h->lev_S[0], -1.0, st))) return rc;   // w = L z_j
            for (int i = 0; i <= j; ++i) Hij(i, j) = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                HIPCHK(launch_multidot(V, len, j + 1, w, len, h->kpart, h->kc, st));
                HIPCHK(hipMemcpyAsync(h->khost, h->kc, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i <= j; ++i) {
                    Hij(i, j) += h->khost[i];
                    h->khost[i] = -h->khost[i];
                }
                HIPCHK(hipMemcpyAsync(h->kc, h->khost, sizeof(double) * (j + 1), hipMemcpyHostToDevice, st));
                HIPCHK(launch_multiaxpy(V, len, j + 1, h->kc, 1.0, w, len, st));
            }
            double hn = 0.0;
            if ((rc = read_norm(h, w, len, st, &hn))) return rc;
            Hij(j + 1, j) = hn;
            if (hn > 0.0) HIPCHK(launch_multiaxpy(V, len, 0, h->kc, 1.0 / hn, w, len, st));
            // apply the previous rotations to column j, then a new one
            for (int i = 0; i < j; ++i) {
                const double a = Hij(i, j), b = Hij(i + 1, j);
                Hij(i, j) = cs[i] * a + sn[i] * b;
                Hij(i + 1, j) = -sn[i] * a + cs[i] * b;
            }
            const double a = Hij(j, j), b = Hij(j + 1, j);
            const double r = std::hypot(a, b);
            cs[j] = r > 0 ? a / r : 1.0;
            sn[j] = r > 0 ? b / r : 0.0;
            Hij(j, j) = r;
            Hij(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            jn = j + 1;
            if (std::fabs(g[j + 1]) <= rtol * fn || hn == 0.0) break;
        }
        // y = R^{-1} g, u += Z y
        for (int i = jn - 1; i >= 0; --i) {
            double v = g[i];
            for (int k = i + 1; k < jn; ++k) v -= Hij(i, k) * y[k];
            y[i] = v / Hij(i, i);
        }
        for (int i = 0; i < jn; ++i) h->khost[i] = y[i];
        HIPCHK(hipMemcpyAsync(h->kc, h->khost, sizeof(double) * jn, hipMemcpyHostToDevice, st));
        HIPCHK(launch_multiaxpy(Z, len, jn, h->kc, 1.0, u, len, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (iters) *iters = it;
    if (relres) *relres = rn / fn;
    if (!std::isfinite(rn)) return fail(STH_ENOCONV, "residual is not finite");
    if (rn > rtol * fn) return fail(STH_ENOCONV, "maxit reached");
    return STH_OK;
}

int sth_speculate(sth_handle* h, int enable) {
    if (!h) return fail(STH_EINVAL, "null handle");
    h->speculate = enable != 0;
    return STH_OK;
}

int sth_use_graphs(sth_handle* h, int enable) {
    if (!h) return fail(STH_EINVAL, "null handle");
    h->use_graph = enable != 0;
    if (!h->use_graph) drop_graph(h);
    return STH_OK;
}

int sth_restrict(sth_handle* h, int level, const double* r, double* rc, void* stream) {
    sth_handle* o = h && r && rc ? level_owner(h, level) : nullptr;
    if (!o || (level + 1 >= o->L && !o->child)) return fail(STH_EINVAL, "bad argument");
    if (level + 1 == o->L) {
        if (r == o->buf0 || rc == o->buf0 || rc == o->buf1) return fail(STH_EINVAL, "vector aliases a workspace");
        return restrict_space(o, r, rc, (hipStream_t)stream);
    }
    return restrict_lvl(o, level, r, rc, (hipStream_t)stream);
}

int sth_prolong_add(sth_handle* h, int level, const double* ec, double* u, void* stream) {
    sth_handle* o = h && ec && u ? level_owner(h, level) : nullptr;
    if (!o || (level + 1 >= o->L && !o->child)) return fail(STH_EINVAL, "bad argument");
    if (level + 1 == o->L) return prolong_space(o, ec, u, (hipStream_t)stream);
    return prolong_lvl(o, level, ec, u, (hipStream_t)stream, o->Nx);
}

int sth_norm(sth_handle* h, const double* v, double* out, void* stream) {
    if (!h || !v || !out) return fail(STH_EINVAL, "null argument");
    return read_norm(h, v, h->lev_S[0] * slab_len(h), (hipStream_t)stream, out);
}

int sth_destroy(sth_handle* h) {
    if (!h) return STH_OK;
    // graph first: its nodes reference the buffers below
    drop_graph(h);
    if (h->child) sth_destroy(h->child);
    for (void* q : {(void*)h->rj0, (void*)h->pj0, (void*)h->rco, (void*)h->pco, (void*)h->cf, (void*)h->cu,
                    (void*)h->mrst})
        if (q) (void)hipFree(q);
    for (double* q : h->mr)
        if (q) (void)hipFree(q);
    double* ptrs[] = {h->Tf, h->Ti, h->mu1, h->M1b, h->K1b, h->buf0, h->buf1, h->partial, h->dnorm, h->dktmt,
                      h->Cf, h->Ci, h->Gf, h->e0, h->e1, h->e2, h->e3, h->cpartial, h->kv, h->kz, h->kc,
                      h->kpart, h->vw};
    for (double* q : ptrs)
        if (q) (void)hipFree(q);
    for (auto* vec : {&h->lu, &h->lf, &h->lu2, &h->eu, &h->ef, &h->eu2})
        for (double* q : *vec)
            if (q) (void)hipFree(q);
    if (h->hnorm) (void)hipHostFree(h->hnorm);
    if (h->hflag) (void)hipHostFree(h->hflag);
    if (h->hseq) (void)hipHostFree(h->hseq);
    if (h->dthr) (void)hipFree(h->dthr);
    if (h->dmix) (void)hipFree(h->dmix);
    if (h->dgo) (void)hipFree(h->dgo);
    for (auto e : h->evring)
        if (e) (void)hipEventDestroy(e);
    if (h->khost) (void)hipHostFree(h->khost);
    for (auto e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return STH_OK;
}

int sth_timing(sth_handle* h, unsigned class_mask) {
    if (!h) return fail(STH_EINVAL, "null handle");
    if (class_mask) {
        // wait for outstanding records before their events are reused
        for (auto& r : h->recs) (void)hipEventSynchronize(r.b);
        h->recs.clear();
        drop_graph(h);
        h->pool_used = 0;
        for (int c = 0; c < STH_K_COUNT; ++c) {
            h->gms[c] = h->gfl[c] = h->gby[c] = 0.0;
            h->gcnt[c] = 0;
        }
    }
    h->timing = class_mask != 0;
    h->timing_mask = class_mask;
    return h->child ? sth_timing(h->child, class_mask) : STH_OK;
}

int sth_timing_level(sth_handle* h, int level) {
    if (!h || level < -1 || level >= sth_num_levels(h)) return fail(STH_EINVAL, "bad argument");
    // level made local to the handle of the chain that holds it; the others
    // record nothing
    int rest = level;                   // local to the current handle; -1 once placed
    for (sth_handle* o = h; o; o = o->child) {
        if (level < 0) {
            o->timing_level = -1;
        } else if (rest >= 0 && rest < o->L) {
            o->timing_level = rest;
            rest = -1;
        } else {
            o->timing_level = 1 << 30;
            if (rest >= 0) rest -= o->L;
        }
    }
    return STH_OK;
}

int sth_timing_report(sth_handle* h, int kclass, int* launches, double* ms, double* flops, double* bytes) {
    if (!h || kclass < 0 || kclass >= STH_K_COUNT) return fail(STH_EINVAL, "bad argument");
    int cnt = h->gcnt[kclass];
    double t = h->gms[kclass], fl = h->gfl[kclass], by = h->gby[kclass];
    for (auto& r : h->recs) {
        if (r.cls != kclass) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(STH_EHIP, "event sync");
        float e = 0;
        if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return fail(STH_EHIP, "event time");
        ++cnt;
        t += e;
        fl += r.flops;
        by += r.bytes;
    }
    if (h->child) {
        int c2 = 0;
        double t2 = 0, f2 = 0, b2 = 0;
        const int rc = sth_timing_report(h->child, kclass, &c2, &t2, &f2, &b2);
        if (rc) return rc;
        cnt += c2;
        t += t2;
        fl += f2;
        by += b2;
    }
    if (launches) *launches = cnt;
    if (ms) *ms = t;
    if (flops) *flops = fl;
    if (bytes) *bytes = by;
    return STH_OK;
}

// ---- host introspection ----------------------------------------------------
int sth_host_factors(const sth_problem* p, int level, sth_factors* out) {
    if (!p || !out) return fail(STH_EINVAL, "null argument");
    Problem q = to_problem(p);
    Setup S;
    std::string e;
    int st = build_setup(q, S, e);
    if (st != 0) return fail(st, e);
    if (level < 0 || level >= (int)S.levels.size()) return fail(STH_EINVAL, "bad level");
    int n = S.n, Nt = S.Nt;
    out->n = n;
    out->N_t = Nt;
    out->n_levels = (int)S.levels.size();
    const TemporalLevel& L = S.levels[level];
    out->cond_V = L.condV;
    auto cp = [](double* dst, const std::vector<double>& src) {
        if (dst) std::memcpy(dst, src.data(), src.size() * sizeof(double));
    };
    cp(out->M1, S.M1.a);
    cp(out->K1, S.K1.a);
    cp(out->U, S.U.a);
    cp(out->mu, S.mu);
    cp(out->Kt, L.Kt.a);
    cp(out->Mt, L.Mt.a);
    if (L.Pt.r > 0) cp(out->Pt, L.Pt.a);
    cp(out->V, L.V.a);
    cp(out->W, L.W.a);
    cp(out->eig_re, L.re);
    cp(out->eig_im, L.im);
    out->schur = L.schur ? 1 : 0;
    if (L.schur) cp(out->R, L.R.a);
    if (out->mode_weights) cp(out->mode_weights, residual_mode_weights(S));
    return STH_OK;
}

int sth_host_space_prolongation(int n_elem_c, int degree, double* out) {
    if (!out || n_elem_c < 1 || degree < 1 || degree > kMaxDeg || n_elem_c + degree - 2 < 1)
        return fail(STH_EINVAL, "bad argument");
    Mat Px;
    space_prolongation(n_elem_c, degree, Px);
    std::memcpy(out, Px.a.data(), sizeof(double) * Px.a.size());
    return STH_OK;
}

int sth_host_load_1d(const sth_problem* p, double omega, double phase, int k, double* time_part,
                     double* space_part) {
    if (!p) return fail(STH_EINVAL, "null argument");
    Problem q = to_problem(p);
    std::string e = validate(q);
    if (!e.empty()) return fail(STH_EINVAL, e);
    std::vector<double> tmp;
    if (time_part) {
        load_time(q, omega, phase, tmp);
        std::memcpy(time_part, tmp.data(), tmp.size() * sizeof(double));
    }
    if (space_part) {
        load_space(q, k, tmp);
        std::memcpy(space_part, tmp.data(), tmp.size() * sizeof(double));
    }
    return STH_OK;
}

}  // extern "C"
