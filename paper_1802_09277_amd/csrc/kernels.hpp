// Launchers of the gfx950 kernels.  All pointers are device pointers; every
// launcher returns the HIP error of its launch.  Vectors use the layout
// v[slab][t][z][y][x] (x fastest); n is the number of interior spline
// functions per spatial axis, np = n rounded up to a multiple of 16.
#pragma once
#include <hip/hip_runtime.h>

namespace sth {

constexpr int kNt = 8;          // maximum time functions per slab

struct TimeOp {                 // residual: temporal matrices of the level
    double Kt[kNt * kNt];
    double Mt[kNt * kNt];
};
struct TimeMix {                // slab inverse: temporal decomposition of the level
    double W[kNt * kNt];
    double V[kNt * kNt];
    // eigen form (schur == 0): A^{-1} = V (Z + mu I)^{-1} W with Z block
    // diagonal in fixed 2x2 blocks (rows 2j, 2j+1; a complex pair
    // [[a, b], [-b, a]] or two real eigenvalues) and a trailing 1x1 block
    // when Nt is odd; zd[k] = Z[k][k], zo[k] = the other entry of row k in
    // its block (0 for a 1x1 block)
    double zd[kNt];
    double zo[kNt];
    int kind[kNt];              // Schur form: 0 1x1 block, 1 first row of a 2x2 block, 2 second row
    int schur;                  // 1: (R + mu I) y = W g by block back substitution
    double R[kNt * kNt];        // real Schur form (quasi upper triangular)
};
struct Transfer {               // 2Nt x Nt prolongation
    double P[2 * kNt * kNt];
};

// Guards of speculatively enqueued multigrid cycles: the launches of such a
// cycle take a device int and return at once when it holds 0.  The final sum
// of a cycle-close pass with a CycleFlag stores 1 there (and in the mapped
// host copy) when the lower bound of its B-spline residual,
// max(nb_lo ||r^||^2, (1 - 1e-8) sum_m v_m r^_m^2), exceeds *thr =
// (rtol ||f||)^2, and 0 otherwise (possible convergence, or non-finite); a
// skipped sum stores 0.
// With exact = 1 (sum of an exact B-spline norm) the flag is instead 1 when
// the host will end the solve on it: ||r|| = sqrt(sum) is not finite or not
// above thr[1] = rtol ||f||.
struct CycleFlag {
    int* dev = nullptr;
    int* host = nullptr;           // mapped pinned host memory (may be null)
    const double* thr = nullptr;   // device pair: (rtol ||f||)^2, rtol ||f||
    double nb_lo = 0.0;
    int exact = 0;
    // completion mark: after the outputs above, a system-scope fence and
    // *seq = seq_val (mapped host memory) for a host that polls instead of
    // waiting for an event
    int* seq = nullptr;
    int seq_val = 0;
};

// r = f + sign * (-(A u)_n + (B u)_{n-1}) for slabs [s0, s0+ns) of a vector
// with slab length Nt*n^dim; the coupling uses slab s-1 of the same vector
// when s > 0.  f may be null (treated as zero).  M1b/K1b: bands [n][2p+1];
// ktmt: device copy of op (K_t then M_t, kNt x kNt each).
hipError_t launch_residual(int dim, int Nt, int p, int n, const double* M1b, const double* K1b,
                           const TimeOp& op, const double* ktmt, const double* f, const double* u, double* r,
                           long s0, long ns, double sign, hipStream_t st);

// The residual with its squared norm (2-D images of 128 or more columns and
// small degrees: residual_norm_fused): r = f - L u over all ns slabs, and
// sum r^2 to out[0]
// (and out_host, mapped pinned host memory, if not null) in a fixed order;
// partial needs as many entries as the residual kernel has blocks (at most
// max_partial).
bool residual_norm_fused(int dim, int n, int p, int Nt);
hipError_t launch_residual_norm(int dim, int Nt, int p, int n, const double* M1b, const double* K1b,
                                const double* ktmt, const double* f, const double* u, double* r, long ns,
                                double* partial, long max_partial, double* out, double* out_host, hipStream_t st);

// out[line][j] (EPI) sum_k in[line][k] T[k][j] for `lines` contiguous lines
// of length n.  EPI 0: store, 1: out += alpha*acc, 2: out = alpha*acc.
// prec (sth_prec): 0 MFMA f64, 1 MFMA f32 (FP32 accumulation), 2 BF16x3.
hipError_t launch_xform_x(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                          long lines, double alpha, hipStream_t st, const int* guard = nullptr, int sym = 0,
                          int io = 0);
// the panel form of launch_xform_x with float data on one side (reduced
// precisions, np <= 256): io 2 writes float output (the intermediate of a
// forward transform), 1 reads float input (that of an inverse transform)
hipError_t launch_xform_panel_x_io(int prec, int epi, const double* in, double* out, const double* T, int n, int np,
                                   long lines, double alpha, hipStream_t st, const int* guard, int sym, int io);

// Strided axis: in[b][k][i] (k stride `inner`), out[b][j][i] = sum_k T[k][j] in[b][k][i].
hipError_t launch_xform_s(int prec, const double* in, double* out, const double* T, int n, int np,
                          long nbatch, long inner, hipStream_t st, const int* guard = nullptr, int io_f32 = 0,
                          int sym = 0);
// sym 1 (forward) and 2 (inverse): T's modes split into even ones [0, n/2)
// and odd ones [n/2, n) under the reflection i -> n-1-i, which halves the
// multiply-adds; only for n = np with xform_split_supported(n)
bool xform_split_supported(int n);
// (both per-axis launchers: every block returns at once when guard is given
// and *guard == 0, as in the guards of speculative cycles; launch_xform_s
// with io_f32 2 writes float output, 1 reads float input, 3 both (reduced
// precisions), for np <= 256 a multiple of 32: xform_panel_f32_io(np))
bool xform_panel_f32_io(int np);

// Both spatial axes of 2-D images (n x n each, nimg images, image i at
// in + i ldi and out + i ldo; 0: n^2) in one kernel:
// dir 0: out = U^T R U; dir 1: Z = U Y U^T with epilogue epi (0 store,
// 1 out += alpha Z, 2 out = alpha Z).  Upad is U padded to np x np; prec 0
// computes in FP64 (MFMA f64), 1 in FP32 (MFMA f32, FP32 accumulation).
constexpr int kXform2dMaxNp = 96;
bool xform2d_supported(int np);
// Spatial modes per time row of an eigenbasis vector: n^d, padded to a
// multiple of 16 (128-byte rows) on the 2-D path of the one-kernel
// transforms; the padded modes hold zeros (every eigenbasis kernel maps zero
// data of a mode to zero).  The eigenbasis launchers use this count.
long eig_modes(int dim, int n);
// io_f32 (FP32 transforms only): 2 writes float output (out addresses float
// data), 1 reads float input
hipError_t launch_xform2d(int prec, int dir, int epi, const double* in, double* out, const double* Upad, int n, int np,
                          long nimg, double alpha, hipStream_t st, const int* guard = nullptr, long ldi = 0,
                          long ldo = 0, int io_f32 = 0);

// BF16x3 form of the same: out = M (In M^T) per image with the products
// accumulated in FP32 from hi*hi + hi*lo + lo*hi bf16 MFMA products; pass
// M = U^T (padded) for the forward and M = U for the inverse transform.
// Image strides ldi, ldo (0: n^2) and the guard as in launch_xform2d.
hipError_t launch_xform2d_bf16x3(int epi, const double* in, double* out, const double* Mpad, int n, int np,
                                 long nimg, double alpha, hipStream_t st, const int* guard = nullptr, long ldi = 0,
                                 long ldo = 0, int io_f32 = 0);

// Per slab and spatial mode (nx modes per time row; 0: n^d): out[:, m] = A_m^{-1} in[:, m], A_m^{-1} =
// V (Z + mu_m I)^{-1} W (or the real Schur form of the level).  fwdsub:
// instead the exact solution of the S coupled slabs in the eigenbasis,
// out_s = A_m^{-1}(in_s + e_1 out_{s-1}[Nt-1]) (forward substitution),
// computed parallel in time (in and out must differ).
hipError_t launch_timemix(int dim, int Nt, const TimeMix& tm, const double* mu1, int n, long nx,
                          const double* in, double* out, long S, bool fwdsub, hipStream_t st,
                          const int* guard = nullptr, int vt = 0);

// Iteration in the spatial eigenbasis (all pointwise over spatial modes;
// ktmt = device K_t then M_t of the level).  The launchers with a `vt`
// argument take eigenbasis vectors stored in FP64 (vt = 0) or FP32 (vt = 1:
// the vector pointers then address float data); the arithmetic is FP64
// either way:
//  uout = v + omega A^{-1}(fh - L v) with v = uin (+ (P (x) I) ec when ec is
//  not null: the prolonged coarse correction, S/2 coarse slabs); uin is not
//  read when zero_guess (then ec must be null)
hipError_t launch_eig_smooth(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                             const double* fh, const double* uin, double* uout, long S, double omega,
                             bool zero_guess, const double* ec, const Transfer& tr, hipStream_t st,
                             const int* guard = nullptr);
//  descent on a coarse level from a zero guess, one pass over fl (chains of
//  `chain` slabs per thread, chain even and dividing S): uout = omega A^{-1} fl,
//  fc = (P^T (x) I)(fl - L uout) on slab pairs
hipError_t launch_eig_down(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                           const double* fl, double* uout, double* fc, const Transfer& tr, double omega, long S,
                           int chain, hipStream_t st, const int* guard = nullptr, int vt = 0);
//  post-smoothing step of a level whose pre-smoothing step started from zero
//  (so A u = omega f slab by slab), with the prolonged coarse correction
//  (S/2 coarse slabs) added first, in closed form without f or a slab solve:
//  uout = (2 - omega) uin + (1 - omega)(P (x) I) ec + omega q A^{-1} e_1 (q the
//  coupling row of the previous slab of uin + (P (x) I) ec); chains as above
hipError_t launch_eig_post(int dim, int Nt, const TimeMix& tm, const double* mu1, int n, const double* uin,
                           const double* ec, double* uout, const Transfer& tr, double omega, long S, int chain,
                           hipStream_t st, const int* guard = nullptr, int vt = 0);
//  end of a cycle on the finest level, in one pass over f^ and u^ (chains as
//  above): ||fh - L uin||^2 and its lower and upper mode-weighted forms
//  sum_m v_m |r_m|^2, sum_m w_m |r_m|^2 (weights from the per-axis table vw
//  of the diagonal entries and absolute row sums of G = C^T C) to
//  out[0..2], and to out_host[0..2] (mapped pinned host memory) if not null;
//  uout = uin + omega A^{-1}(fh - L uin), fc = (P^T (x) I)(fh - L uout) on
//  slab pairs.  partial needs max_partial >= 3 ceil((S/chain) Nx / 256)
//  entries
hipError_t launch_eig_cycle_end(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                                const double* fh, const double* uin, double* uout, double* fc, const Transfer& tr,
                                double omega, long S, int chain, const double* vw, double* partial,
                                long max_partial, double* out, double* out_host, hipStream_t st,
                                const CycleFlag& flag = CycleFlag{}, int vt = 0, const int* unz = nullptr);
//  (unz given and *unz == 0 on the device: uin is zero and is not read)
//  close of a cycle on the finest level and start of the next in one pass
//  (chains and sums as above): u1 = upre + (P_t (x) I) ec, uend = u1 +
//  omega A^{-1}(fh - L u1) (the cycle's result), the three sums of
//  fh - L uend, unext = uend + omega A^{-1}(fh - L uend), fc =
//  (P^T (x) I)(fh - L unext) on slab pairs; the three iterate buffers differ.
//  uend null: the result is not stored.  unext null (fc and partial null,
//  sums false): the pass stores uend alone, bitwise as the full pass does.
hipError_t launch_eig_cycle_close(int dim, int Nt, const TimeMix& tm, const double* ktmt, const double* mu1, int n,
                                  const double* fh, const double* upre, const double* ec, double* uend,
                                  double* unext, double* fc, const Transfer& tr, double omega, long S, int chain,
                                  const double* vw, double* partial, long max_partial, double* out,
                                  double* out_host, hipStream_t st, const int* guard = nullptr,
                                  const CycleFlag& flag = CycleFlag{}, bool sums = true, int vt = 0);
//  the final sums of a cycle-close pass launched with sums = false (same S,
//  chain, partial, outputs, guard and flag), as a separate launch
hipError_t launch_cycle_sums(int dim, int n, long S, int chain, double* partial, double* out, double* out_host,
                             hipStream_t st, const int* guard = nullptr, const CycleFlag& flag = CycleFlag{});
//  thr[0..1] = (rtol F)^2, rtol F with F = ||f|| (1 if ||f|| = 0), from f2 = ||f||^2
hipError_t launch_spec_threshold(double* thr, const double* f2, double rtol, hipStream_t st);
//  *flag = value, and thr[0..1] = thr_value, thr_lin when thr is not null and thr_value >= 0
hipError_t launch_set_flag(int* flag, int value, hipStream_t st, double* thr = nullptr, double thr_value = -1.0,
                           double thr_lin = -1.0);
//  the two coarsest levels of a V(1,1) cycle in one pass from level a's
//  right-hand side fa (SA slabs; level b has SA/2): smoothing step from zero,
//  restriction of its residual, exact solve of level b, prolongation and the
//  post-smoothing step; ua = level a's result (fa and ua differ).  The
//  per-level slab inverses are device copies, both of the same form (schur).
//  coarse_tail_shape says whether SA fits (slab groups of 2..8 level-a slabs).
bool coarse_tail_shape(int Nt, long SA, int* G, int* LA);
hipError_t launch_eig_coarse_tail(int dim, int Nt, const TimeMix* tma_dev, const TimeMix* tmb_dev, bool schur,
                                  const double* mu1, int n, const double* fa, double* ua,
                                  const Transfer& tr, double omega, long SA, hipStream_t st,
                                  const int* guard = nullptr, int vt = 0);
//  the three coarsest levels in one pass (a, b, c with SA, SA/2, SA/4
//  slabs): the descent of the two-level pass on a and on b, the exact solve
//  of c, and the closed-form post-smoothing step on b and then on a; ua =
//  level a's result.  coarse_tail3_shape says whether SA fits (slab groups
//  of 4 or 8 level-a slabs; 64 groups for N_t <= 3).
bool coarse_tail3_shape(int Nt, long SA, int* G, int* LA);
hipError_t launch_eig_coarse_tail3(int dim, int Nt, const TimeMix* tma_dev, const TimeMix* tmb_dev,
                                   const TimeMix* tmc_dev, bool schur, const double* mu1, int n, const double* fa,
                                   double* ua, const Transfer& tr, double omega, long SA, hipStream_t st,
                                   const int* guard = nullptr, int vt = 0);
//  rh = fh - L uh
hipError_t launch_eig_residual(int dim, int Nt, const double* ktmt, const double* mu1, int n, const double* fh,
                               const double* uh, double* rh, long S, hipStream_t st);
//  fc = (P^T (x) I)(fh - L uh) on slab pairs
hipError_t launch_eig_resid_restrict(int dim, int Nt, const Transfer& tr, const double* ktmt, const double* mu1,
                                     int n, const double* fh, const double* uh, double* fc, long Sc,
                                     hipStream_t st);

//  out[0] = sum over the nimg n x n images Y (image i at in + i ldi; 0: n^2)
//  of ||C Y C^T||_F^2 (2-D, np <= 96),
//  the squared B-spline norm of an eigenbasis vector without forming it,
//  computed as <Y G, G Y>_F with Gpad = C^T C (np x np, zero padded); partial
//  needs max_blocks entries; the sum also goes to out_host (mapped pinned host
//  memory) if not null
hipError_t launch_gram_norm2d(const double* in, const double* Gpad, int n, int np, long nimg, double* partial,
                              int max_blocks, double* out, double* out_host, hipStream_t st,
                              const CycleFlag& flag = CycleFlag{}, long ldi = 0);

// rc[m] = (P^T (x) I) [r[2m]; r[2m+1]],  m < Sc
hipError_t launch_restrict(int Nt, const Transfer& tr, const double* r, double* rc, long Sc,
                           long Nx, hipStream_t st);
// u[2m..2m+1] += (P (x) I) e[m]
hipError_t launch_prolong(int Nt, const Transfer& tr, const double* e, double* u, long Sc,
                          long Nx, hipStream_t st);
// out[o][i][c] = sum_{k<W} coef[i W + k] in[o][j0[i] + k][c] over [outer][n_in][inner]
hipError_t launch_band_axis(const double* in, double* out, long outer, int n_in, int n_out, long inner,
                            const int* j0, const double* coef, int W, hipStream_t st);

// ---- MinRes slab inverse (Theorems 3.8, 3.10) ------------------------------
constexpr int kMrState = 13;    // doubles of MinRes state per (slab, pair) system
struct TimeRowMix {             // out row t = sout[t] sum_t' M[t][t'] sin[t'] in row t'
    double M[kNt * kNt];
    double sin[kNt];
    double sout[kNt];
};
struct PairOps {                // A_bar of the pairs (rows 2k, 2k+1 of a slab)
    int npairs;
    double alpha[kNt / 2];
    double a11[kNt / 2], a12[kNt / 2], a21[kNt / 2], a22[kNt / 2];
};
struct PinvRows {               // P^{-1} per time row: scale / (mu + shift) in the eigenbasis
    double scale[kNt];
    double shift[kNt];
};
hipError_t launch_time_mix(const double* in, double* out, const TimeRowMix& m, long ns, int nt, long nx, int epi,
                           double alpha, hipStream_t st);
hipError_t launch_pair_apply(int dim, const double* z, double* q, const double* M1b, const double* K1b, int n, int p,
                             long ns, int nt, const PairOps& ops, hipStream_t st);
hipError_t launch_pinv_scale(double* t, long ns, int nt, long nx, int dim, const double* mu1, int n,
                             const PinvRows& pr, hipStream_t st);
// which 0: q.z into the state's slot, 1: v.z
hipError_t launch_pair_dot(const double* a, const double* b, double* state, int which, long ns, int nt, int npairs,
                           long nx, hipStream_t st);
hipError_t launch_minres_init(double* state, long nsys, hipStream_t st);
hipError_t launch_lanczos(const double* q, const double* vc, const double* vp, double* vn, const double* state,
                          long ns, int nt, int npairs, long nx, hipStream_t st);
hipError_t launch_minres_scalars(double* state, long nsys, hipStream_t st);
hipError_t launch_minres_update(const double* zc, const double* w1, double* w2, double* y, const double* state,
                                long ns, int nt, int npairs, long nx, hipStream_t st);
hipError_t launch_pair_split(double* y, double* zc, double* w1, double* w2, double* vp, long ns, int nt, int npairs,
                             long nx, hipStream_t st);

// v[0..len) = val, skipped when skip is given and *skip != 0 (f32: v
// addresses float data)
hipError_t launch_fill(double* v, long len, double val, hipStream_t st, const int* skip = nullptr, int f32 = 0);
// *flag = 1 if some entry of v[0..len) is not zero (NaN included), else 0
hipError_t launch_any_nonzero(const double* v, long len, int* flag, hipStream_t st);

// Krylov vectors V_i = V + i*ld (i < k <= kMaxKrylov), for the FGMRES loop:
//  out[i] = <V_i, w> (deterministic; partial needs 1024 * kMaxKrylov entries)
//  w = alpha w + sum_i c[i] V_i (c: k device values)
constexpr int kMaxKrylov = 32;
hipError_t launch_multidot(const double* V, long ld, int k, const double* w, long len, double* partial, double* out,
                           hipStream_t st);
hipError_t launch_multiaxpy(const double* V, long ld, int k, const double* c, double alpha, double* w, long len,
                            hipStream_t st);

// Two-stage deterministic sum of squares: partial sums over a fixed number
// of blocks, then one block; result in out[0].
constexpr int kNormBlocks = 1024;
hipError_t launch_norm2(const double* v, long len, double* partial, double* out, hipStream_t st);

// f[s][t][z][y][x] = sum_m T[m][s*Nt+t] * X[m][0][x] * X[m][1][y] (* X[m][2][z])
hipError_t launch_rhs(int dim, int Nt, int n, int n_modes, const double* Tpart, const double* Xpart,
                      double* f, long S, hipStream_t st);

}  // namespace sth
