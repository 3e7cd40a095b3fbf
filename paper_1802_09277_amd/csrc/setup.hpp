// Host FP64 setup of the space-time slab solver: 1-D B-spline matrices,
// temporal pencils per multigrid level, their decompositions and guards.
// Pure C++ (no HIP); the runtime uploads the results.
#pragma once
#include <complex>
#include <string>
#include <vector>

namespace sth {

constexpr int kMaxNt = 8;     // N_t = n_elem_t + degree supported by the kernels
constexpr int kMaxDeg = 4;

struct Mat {
    int r = 0, c = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int rows, int cols) : r(rows), c(cols), a(size_t(rows) * cols, 0.0) {}
    double& operator()(int i, int j) { return a[size_t(i) * c + j]; }
    double operator()(int i, int j) const { return a[size_t(i) * c + j]; }
};

// ---- splines ---------------------------------------------------------------
// Open uniform knot vector on [a,b] with n_el elements of degree p.
std::vector<double> open_knots(double a, double b, int n_el, int p);
// Gauss-Legendre nodes and weights on [-1,1] (Newton on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);
// Nonzero B-splines of degree p at x in knot span `span` (t[span] <= x <
// t[span+1]) and their first derivatives: values/derivs[r] belong to basis
// function span-p+r.
void basis_local(const std::vector<double>& t, int p, int span, double x,
                 double* values, double* derivs);
int find_span(const std::vector<double>& t, int p, double x);

// ---- small dense linear algebra ----------------------------------------------
bool lu_inverse(const Mat& A, Mat& inv);                      // partial pivoting
bool lu_solve_inplace(Mat A, std::vector<double>& b);
bool cholesky(const Mat& A, Mat& L);
void sym_eigen(const Mat& A, std::vector<double>& evals, Mat& evecs);   // A symmetric
// Eigenvalues and eigenvectors of a real nonsymmetric matrix (small).
bool nonsym_eigen(const Mat& A, std::vector<std::complex<double>>& lam,
                  std::vector<std::vector<std::complex<double>>>& vecs);
double cond2(const Mat& A);                                   // sigma_max / sigma_min
// Real Schur form A = Q T Q^T of a small matrix: Q orthogonal, T upper
// quasi-triangular (1x1 and 2x2 diagonal blocks).  false if QR stalls.
bool real_schur(const Mat& A, Mat& T, Mat& Q);

// ---- problem quantities ------------------------------------------------------
struct Problem {
    int dim, n_elem, degree, n_slabs, n_elem_t;
    double T, theta, omega;
    int nu_pre, nu_post, prec;
    int coarse_slabs;
    int basis;
    int temporal = 2;      // 0 diagonalisation, 1 real Schur, 2 automatic
    double space_ratio = 0.0;   // > 0: coarsen in space too where tau_l / h_l^2 >= space_ratio
    int level_cap = 0;     // > 0: at most this many levels of this spatial mesh
    int minres_iters = 0;  // > 0: smoother slab inverse by this many MinRes iterations per pair
    int n() const { return n_elem + degree - 2; }
    int Nt() const { return n_elem_t + degree; }
    double tau() const { return T / n_slabs; }
    double sigma() const { return theta * tau() / n_elem_t; }
};

struct TemporalLevel {
    int S = 0;             // slabs on this level
    double tau = 0;        // slab length
    Mat Kt, Mt;            // eq. TimeMatrices with the finest sigma
    Mat Pt;                // 2Nt x Nt prolongation to the next coarser level
    Mat V, W;              // real block eigenvectors, W = (Mt V)^{-1}; Schur: V = Q, W = Q^T Mt^{-1}
    std::vector<double> re, im;   // eigen pairs (im = +b,-b on a pair)
    std::vector<int> kind;        // 0 real / 1x1 block, 1 first of a pair / 2x2 block, 2 second
    double condV = 0;             // of the eigenvector matrix (also computed for the Schur form)
    bool schur = false;           // W K_t V = R quasi-triangular (else block diagonal)
    Mat R;                        // Schur form: R = Q^T Mt^{-1} Kt Q
};

struct Setup {
    Problem prob;
    int n = 0, Nt = 0;
    Mat M1, K1, U;         // 1-D spatial matrices (interior), eigenvectors
    std::vector<double> mu;
    // n / 2 when n is even and the pencil is symmetric under the reflection
    // i -> n - 1 - i: then columns [0, half) of U are even and [half, n) odd
    // (each block in ascending mu); 0 otherwise
    int half = 0;
    double m1_min = 0, m1_max = 0;   // extreme eigenvalues of M1 (eigenbasis iteration only)
    std::vector<TemporalLevel> levels;
};

// Levels of the finest spatial mesh when the hierarchy coarsens in space
// and time at their last transition (tau_l / h_l^2 >= space_ratio with an
// even number of elements, at least 4, per axis); 0 when it coarsens in time
// only.  The levels below belong to the problem on the halved mesh.
int space_transition(const Problem& p);

// Validates the problem; returns an error message or "".
std::string validate(const Problem& p);
// Full setup.  status: 0 ok, -4 not positive, -5 ill-conditioned, -1 invalid.
int build_setup(const Problem& p, Setup& s, std::string& err);

// Per 1-D mode j of the spatial eigenbasis: G_jj and sum_k |G_jk| of
// G = C^T C, C = M1 U (2n entries, interleaved), the weights of the lower
// bound x^T (G (x) .. (x) G) x >= sum_m (2 prod G_jj - prod sum_k |G_jk|) x_m^2.
std::vector<double> residual_mode_weights(const Setup& s);

// Spatial 1-D matrices (interior functions), banded with bandwidth p.
void space_matrices(int n_elem, int p, Mat& M1, Mat& K1);
// Temporal matrices on a slab of length tau with n_el elements and SUPG sigma.
void time_matrices(double tau, int n_el, int p, double sigma, Mat& Kt, Mat& Mt);
// Prolongation coarse slab (length 2 tau) -> two fine slabs by knot insertion.
void time_prolongation(int n_el, int p, Mat& Pt);
// Prolongation of the interior spatial functions, coarse mesh of n_elem_c
// elements -> fine mesh of 2 n_elem_c elements on (0,1), by knot insertion
// ((n_f x n_c), banded: p+2 fine functions per coarse one).
void space_prolongation(int n_elem_c, int p, Mat& Px);
// 1-D load vectors of one separable mode.
void load_time(const Problem& p, double omega, double phase, std::vector<double>& out);
void load_space(const Problem& p, int k, std::vector<double>& out);

}  // namespace sth
