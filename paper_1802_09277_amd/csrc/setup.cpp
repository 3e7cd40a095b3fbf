// Host FP64 setup: splines, small dense linear algebra, temporal pencils.
//
// Discretisation (Sections 2.1-2.3): open uniform B-spline bases in space
// and per time slab; spatial 1-D mass/stiffness matrices over the interior
// functions (u = 0 on the lateral boundary); temporal matrices of eq.
// TimeMatrices with the SUPG test function psi + sigma psi' and the upwind
// point term at the start of the slab; sigma = theta * h_t with h_t the
// temporal element size.  Decomposition of the temporal pencil (Sections
// 3.2-3.3): K_t z = lambda M_t z, written in real block form K_t V = M_t V Z
// with Z block diagonal (lambda for a real eigenvalue, [[a, b], [-b, a]] for
// a pair a +- ib), W = (M_t V)^{-1} (the matrix Y of eq.
// equ:ST:generalDecompA), with the a-posteriori check Re(lambda) > 0 of
// Section 3.2 and a guard on cond(V) (Section 3.3, Table 1).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <sstream>

namespace sth {

// ---------------------------------------------------------------------------
// splines
// ---------------------------------------------------------------------------
std::vector<double> open_knots(double a, double b, int n_el, int p) {
    std::vector<double> t;
    for (int i = 0; i <= p; ++i) t.push_back(a);
    for (int k = 1; k < n_el; ++k) t.push_back(a + (b - a) * double(k) / n_el);
    for (int i = 0; i <= p; ++i) t.push_back(b);
    return t;
}

void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
    // Newton iteration on the Legendre polynomial P_q, three-term recurrence
    // for P_q and its derivative; symmetric nodes.
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (q + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (q == 1) { p1 = z; p0 = 1.0; }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= q; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (q == 1) { p1 = z; p0 = 1.0; }
        dp = q * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[q - 1 - i] = z;
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        w[i] = wi;
        w[q - 1 - i] = wi;
    }
    if (q % 2 == 1) x[q / 2] = 0.0;
}

int find_span(const std::vector<double>& t, int p, double x) {
    int N = int(t.size()) - p - 1;
    if (x >= t[N]) return N - 1;
    if (x <= t[p]) return p;
    int lo = p, hi = N;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x < t[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

void basis_local(const std::vector<double>& t, int p, int span, double x,
                 double* values, double* derivs) {
    // Triangular Cox-de Boor table restricted to the p+1 functions that are
    // nonzero on the span; the degree p-1 row gives the derivatives.
    double N[kMaxDeg + 2] = {1.0};
    double Nlow[kMaxDeg + 2] = {0.0};
    double left[kMaxDeg + 2], right[kMaxDeg + 2];
    if (p == 0) Nlow[0] = 0.0;
    for (int j = 1; j <= p; ++j) {
        if (j == p)
            for (int r = 0; r < p; ++r) Nlow[r] = N[r];   // degree p-1 values
        left[j] = x - t[span + 1 - j];
        right[j] = t[span + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
    for (int r = 0; r <= p; ++r) values[r] = N[r];
    if (!derivs) return;
    if (p == 0) { derivs[0] = 0.0; return; }
    // Nlow[r] is N_{span-p+1+r, p-1}; N'_{i,p} = p N_{i,p-1}/(t_{i+p}-t_i)
    //                                         - p N_{i+1,p-1}/(t_{i+p+1}-t_{i+1})
    for (int r = 0; r <= p; ++r) {
        int i = span - p + r;
        double a = (r >= 1) ? Nlow[r - 1] : 0.0;          // N_{i, p-1}
        double b = (r <= p - 1) ? Nlow[r] : 0.0;          // N_{i+1, p-1}
        double d = 0.0;
        double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
        if (d1 > 0) d += p * a / d1;
        if (d2 > 0) d -= p * b / d2;
        derivs[r] = d;
    }
}

// ---------------------------------------------------------------------------
// dense linear algebra
// ---------------------------------------------------------------------------
static bool lu_factor(Mat& A, std::vector<int>& piv) {
    int n = A.r;
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int pr = k;
        double best = std::fabs(A(k, k));
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A(i, k)) > best) { best = std::fabs(A(i, k)); pr = i; }
        piv[k] = pr;
        if (best == 0.0) return false;
        if (pr != k)
            for (int j = 0; j < n; ++j) std::swap(A(k, j), A(pr, j));
        for (int i = k + 1; i < n; ++i) {
            double l = A(i, k) / A(k, k);
            A(i, k) = l;
            for (int j = k + 1; j < n; ++j) A(i, j) -= l * A(k, j);
        }
    }
    return true;
}

static void lu_apply(const Mat& LU, const std::vector<int>& piv, double* b) {
    int n = LU.r;
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= LU(i, j) * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= LU(i, j) * b[j];
        b[i] /= LU(i, i);
    }
}

bool lu_solve_inplace(Mat A, std::vector<double>& b) {
    std::vector<int> piv;
    if (!lu_factor(A, piv)) return false;
    lu_apply(A, piv, b.data());
    return true;
}

bool lu_inverse(const Mat& A, Mat& inv) {
    Mat LU = A;
    std::vector<int> piv;
    if (!lu_factor(LU, piv)) return false;
    int n = A.r;
    inv = Mat(n, n);
    std::vector<double> col(n);
    for (int j = 0; j < n; ++j) {
        std::fill(col.begin(), col.end(), 0.0);
        col[j] = 1.0;
        lu_apply(LU, piv, col.data());
        for (int i = 0; i < n; ++i) inv(i, j) = col[i];
    }
    return true;
}

bool cholesky(const Mat& A, Mat& L) {
    int n = A.r;
    L = Mat(n, n);
    for (int j = 0; j < n; ++j) {
        double s = A(j, j);
        for (int k = 0; k < j; ++k) s -= L(j, k) * L(j, k);
        if (s <= 0) return false;
        L(j, j) = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double v = A(i, j);
            for (int k = 0; k < j; ++k) v -= L(i, k) * L(j, k);
            L(i, j) = v / L(j, j);
        }
    }
    return true;
}

void sym_eigen(const Mat& Ain, std::vector<double>& evals, Mat& V) {
    // Cyclic Jacobi rotations (Rutishauser's formulation) until the
    // off-diagonal mass is negligible.
    int n = Ain.r;
    Mat A = Ain;
    V = Mat(n, n);
    for (int i = 0; i < n; ++i) V(i, i) = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += A(i, i) * A(i, i);
            for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                double app = A(p, p), aqq = A(q, q);
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                double tau = s / (1.0 + c);
                A(p, p) = app - t * apq;
                A(q, q) = aqq + t * apq;
                A(p, q) = A(q, p) = 0.0;
                for (int r = 0; r < n; ++r) {
                    if (r == p || r == q) continue;
                    double arp = A(r, p), arq = A(r, q);
                    double nrp = arp - s * (arq + tau * arp);
                    double nrq = arq + s * (arp - tau * arq);
                    A(r, p) = A(p, r) = nrp;
                    A(r, q) = A(q, r) = nrq;
                }
                for (int r = 0; r < n; ++r) {
                    double vrp = V(r, p), vrq = V(r, q);
                    V(r, p) = vrp - s * (vrq + tau * vrp);
                    V(r, q) = vrq + s * (vrp - tau * vrq);
                }
            }
        }
    }
    // sort ascending
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A(a, a) < A(b, b); });
    evals.resize(n);
    Mat Vs(n, n);
    for (int k = 0; k < n; ++k) {
        evals[k] = A(idx[k], idx[k]);
        for (int i = 0; i < n; ++i) Vs(i, k) = V(i, idx[k]);
    }
    V = Vs;
}

typedef std::complex<double> cd;

static bool complex_solve(std::vector<cd> A, int n, std::vector<cd>& b) {
    for (int k = 0; k < n; ++k) {
        int pr = k;
        double best = std::abs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (std::abs(A[i * n + k]) > best) { best = std::abs(A[i * n + k]); pr = i; }
        if (best == 0.0) return false;
        if (pr != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[pr * n + j]);
            std::swap(b[k], b[pr]);
        }
        for (int i = k + 1; i < n; ++i) {
            cd l = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= A[i * n + j] * b[j];
        b[i] /= A[i * n + i];
    }
    return true;
}

bool nonsym_eigen(const Mat& A, std::vector<cd>& lam, std::vector<std::vector<cd>>& vecs) {
    // Householder reduction to upper Hessenberg form, then complex QR steps
    // with Wilkinson shifts (Givens rotations) and deflation; eigenvectors by
    // inverse iteration on the original matrix.
    int n = A.r;
    std::vector<cd> H(size_t(n) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) H[i * n + j] = A(i, j);
    for (int k = 0; k < n - 2; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += std::norm(H[i * n + k]);
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        std::vector<cd> v(n, 0.0);
        cd x0 = H[(k + 1) * n + k];
        cd ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cd(1.0);
        for (int i = k + 1; i < n; ++i) v[i] = H[i * n + k];
        v[k + 1] += ph * alpha;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
        if (vn == 0.0) continue;
        // H <- (I - 2 v v^H / vn) H (I - 2 v v^H / vn)
        for (int j = 0; j < n; ++j) {
            cd s = 0.0;
            for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * H[i * n + j];
            s *= 2.0 / vn;
            for (int i = k + 1; i < n; ++i) H[i * n + j] -= v[i] * s;
        }
        for (int i = 0; i < n; ++i) {
            cd s = 0.0;
            for (int j = k + 1; j < n; ++j) s += H[i * n + j] * v[j];
            s *= 2.0 / vn;
            for (int j = k + 1; j < n; ++j) H[i * n + j] -= s * std::conj(v[j]);
        }
    }
    double anorm = 0.0;
    for (auto& z : H) anorm = std::max(anorm, std::abs(z));
    lam.assign(n, 0.0);
    int hi = n - 1;
    int iter = 0;
    while (hi >= 0) {
        if (hi == 0) { lam[0] = H[0]; break; }
        // find the start of the active unreduced block
        int lo = hi;
        while (lo > 0) {
            double s = std::abs(H[lo * n + lo]) + std::abs(H[(lo - 1) * n + lo - 1]);
            if (s == 0) s = anorm;
            if (std::abs(H[lo * n + lo - 1]) <= 1e-16 * s) { H[lo * n + lo - 1] = 0.0; break; }
            --lo;
        }
        if (lo == hi) { lam[hi] = H[hi * n + hi]; --hi; iter = 0; continue; }
        if (++iter > 500) return false;
        // Wilkinson shift from the trailing 2x2 block
        cd a = H[(hi - 1) * n + hi - 1], b = H[(hi - 1) * n + hi];
        cd c = H[hi * n + hi - 1], d = H[hi * n + hi];
        cd tr = a + d, det = a * d - b * c;
        cd disc = std::sqrt(tr * tr / 4.0 - det);
        cd m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
        cd mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
        if (iter % 11 == 10) mu = d + cd(std::abs(H[hi * n + hi - 1]), 0.0);   // exceptional shift
        for (int i = lo; i <= hi; ++i) H[i * n + i] -= mu;
        std::vector<cd> cs(n), sn(n);
        for (int k = lo; k < hi; ++k) {
            cd x = H[k * n + k], y = H[(k + 1) * n + k];
            double r = std::sqrt(std::norm(x) + std::norm(y));
            cd cc = (r == 0) ? cd(1.0) : x / r;
            cd ss = (r == 0) ? cd(0.0) : y / r;
            cs[k] = cc;
            sn[k] = ss;
            // apply G^H = [[conj(c), conj(s)], [-s, c]] to rows k, k+1
            for (int j = k; j < n; ++j) {
                cd u = H[k * n + j], v = H[(k + 1) * n + j];
                H[k * n + j] = std::conj(cc) * u + std::conj(ss) * v;
                H[(k + 1) * n + j] = -ss * u + cc * v;
            }
        }
        for (int k = lo; k < hi; ++k) {
            cd cc = cs[k], ss = sn[k];
            // apply G on the right to columns k, k+1
            for (int i = 0; i <= std::min(hi, k + 1); ++i) {
                cd u = H[i * n + k], v = H[i * n + k + 1];
                H[i * n + k] = u * cc + v * ss;
                H[i * n + k + 1] = -u * std::conj(ss) + v * std::conj(cc);
            }
        }
        for (int i = lo; i <= hi; ++i) H[i * n + i] += mu;
    }
    // eigenvectors by inverse iteration
    vecs.assign(n, std::vector<cd>(n));
    for (int k = 0; k < n; ++k) {
        std::vector<cd> M(size_t(n) * n);
        cd shift = lam[k] + cd(1e-13 * std::max(anorm, 1.0), 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) M[i * n + j] = A(i, j) - (i == j ? shift : cd(0.0));
        std::vector<cd> x(n);
        for (int i = 0; i < n; ++i) x[i] = cd(1.0 + 0.1 * i, 0.01 * i);
        for (int it = 0; it < 4; ++it) {
            if (!complex_solve(M, n, x)) return false;
            double nn = 0.0;
            for (auto& z : x) nn += std::norm(z);
            nn = std::sqrt(nn);
            for (auto& z : x) z /= nn;
        }
        vecs[k] = x;
    }
    return true;
}

// Householder reflector P = I - 2 v v^T (|v| = 1) with P x = -+|x| e_1; false
// when x is zero
static bool householder(const double* x, int m, double* v) {
    double nx = 0.0;
    for (int i = 0; i < m; ++i) nx += x[i] * x[i];
    nx = std::sqrt(nx);
    if (nx == 0.0) return false;
    for (int i = 0; i < m; ++i) v[i] = x[i];
    v[0] += (x[0] >= 0 ? nx : -nx);
    double nv = 0.0;
    for (int i = 0; i < m; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    for (int i = 0; i < m; ++i) v[i] /= nv;
    return true;
}

// T <- P T on rows r0..r0+m-1, columns c0..c1; T <- T P on columns r0..,
// rows q0..q1; Q <- Q P
static void reflect(Mat& T, Mat& Q, const double* v, int m, int r0, int c0, int c1, int q0, int q1) {
    for (int j = c0; j <= c1; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += v[i] * T(r0 + i, j);
        for (int i = 0; i < m; ++i) T(r0 + i, j) -= 2.0 * v[i] * s;
    }
    for (int i = q0; i <= q1; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += T(i, r0 + j) * v[j];
        for (int j = 0; j < m; ++j) T(i, r0 + j) -= 2.0 * s * v[j];
    }
    for (int i = 0; i < Q.r; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += Q(i, r0 + j) * v[j];
        for (int j = 0; j < m; ++j) Q(i, r0 + j) -= 2.0 * s * v[j];
    }
}

bool real_schur(const Mat& A, Mat& T, Mat& Q) {
    const int n = A.r;
    T = A;
    Q = Mat(n, n);
    for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
    double v[3], x[16];
    // Hessenberg form by Householder reflections
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        for (int i = 0; i < m; ++i) x[i] = T(k + 1 + i, k);
        double vv[16];
        if (!householder(x, m, vv)) continue;
        reflect(T, Q, vv, m, k + 1, 0, n - 1, 0, n - 1);
        for (int i = k + 2; i < n; ++i) T(i, k) = 0.0;
    }
    double anorm = 0.0;
    for (double a : T.a) anorm = std::max(anorm, std::fabs(a));
    if (anorm == 0.0) return true;
    const double eps = 1e-15;
    int hi = n - 1, iter = 0;
    while (hi > 0) {
        // deflation: the active block is l..hi
        int l = hi;
        for (; l > 0; --l) {
            double s = std::fabs(T(l - 1, l - 1)) + std::fabs(T(l, l));
            if (s == 0.0) s = anorm;
            if (std::fabs(T(l, l - 1)) <= eps * s) {
                T(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) { hi -= 1; iter = 0; continue; }          // 1x1 block
        if (l == hi - 1) { hi -= 2; iter = 0; continue; }      // 2x2 block
        if (++iter > 60 * n) return false;
        // Francis double shift: the eigenvalues of the trailing 2x2 block
        // (an ad hoc shift every tenth sweep breaks cycles)
        double s, t;
        if (iter % 10 == 0) {
            double w = std::fabs(T(hi, hi - 1)) + std::fabs(T(hi - 1, hi - 2));
            s = 1.5 * w;
            t = w * w;
        } else {
            s = T(hi - 1, hi - 1) + T(hi, hi);
            t = T(hi - 1, hi - 1) * T(hi, hi) - T(hi - 1, hi) * T(hi, hi - 1);
        }
        // first column of (T - a)(T - b) restricted to the active block
        double x0 = T(l, l) * T(l, l) + T(l, l + 1) * T(l + 1, l) - s * T(l, l) + t;
        double y0 = T(l + 1, l) * (T(l, l) + T(l + 1, l + 1) - s);
        double z0 = T(l + 1, l) * T(l + 2, l + 1);
        for (int k = l; k <= hi - 2; ++k) {
            const double xs[3] = {x0, y0, z0};
            if (householder(xs, 3, v)) {
                const int c0 = std::max(l, k - 1);
                reflect(T, Q, v, 3, k, c0, n - 1, 0, std::min(k + 3, hi));
                if (k > l) T(k + 1, k - 1) = T(k + 2, k - 1) = 0.0;
            }
            x0 = T(k + 1, k);
            y0 = T(k + 2, k);
            if (k < hi - 2) z0 = T(k + 3, k);
        }
        const double xs[2] = {x0, y0};
        if (householder(xs, 2, v)) {
            reflect(T, Q, v, 2, hi - 1, hi - 2, n - 1, 0, hi);
            T(hi, hi - 2) = 0.0;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j + 1 < i; ++j) T(i, j) = 0.0;
    return true;
}

double cond2(const Mat& A) {
    int n = A.c;
    Mat G(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < A.r; ++k) s += A(k, i) * A(k, j);
            G(i, j) = s;
        }
    std::vector<double> ev;
    Mat Q;
    sym_eigen(G, ev, Q);
    if (ev.front() <= 0) return INFINITY;
    return std::sqrt(ev.back() / ev.front());
}

// ---------------------------------------------------------------------------
// matrices of the discretisation
// ---------------------------------------------------------------------------
void space_matrices(int n_elem, int p, Mat& M1, Mat& K1) {
    std::vector<double> t = open_knots(0.0, 1.0, n_elem, p);
    int N = n_elem + p;
    Mat M(N, N), K(N, N);
    std::vector<double> gx, gw;
    gauss_legendre(p + 1, gx, gw);
    double v[kMaxDeg + 1], d[kMaxDeg + 1];
    for (int e = 0; e < n_elem; ++e) {
        int span = e + p;
        double a = t[span], b = t[span + 1];
        for (int q = 0; q <= p; ++q) {
            double x = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
            double w = 0.5 * (b - a) * gw[q];
            basis_local(t, p, span, x, v, d);
            for (int i = 0; i <= p; ++i)
                for (int j = 0; j <= p; ++j) {
                    M(e + i, e + j) += w * v[i] * v[j];
                    K(e + i, e + j) += w * d[i] * d[j];
                }
        }
    }
    int n = N - 2;
    M1 = Mat(n, n);
    K1 = Mat(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            M1(i, j) = M(i + 1, j + 1);
            K1(i, j) = K(i + 1, j + 1);
        }
}

void time_matrices(double tau, int n_el, int p, double sigma, Mat& Kt, Mat& Mt) {
    std::vector<double> t = open_knots(0.0, tau, n_el, p);
    int N = n_el + p;
    Kt = Mat(N, N);
    Mt = Mat(N, N);
    std::vector<double> gx, gw;
    gauss_legendre(p + 1, gx, gw);
    double v[kMaxDeg + 1], d[kMaxDeg + 1];
    for (int e = 0; e < n_el; ++e) {
        int span = e + p;
        double a = t[span], b = t[span + 1];
        for (int q = 0; q <= p; ++q) {
            double x = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
            double w = 0.5 * (b - a) * gw[q];
            basis_local(t, p, span, x, v, d);
            for (int i = 0; i <= p; ++i) {
                double test = v[i] + sigma * d[i];
                for (int j = 0; j <= p; ++j) {
                    Kt(e + i, e + j) += w * d[j] * test;
                    Mt(e + i, e + j) += w * v[j] * test;
                }
            }
        }
    }
    // upwind term psi_j(t_{n-1}) psi_i(t_{n-1}) at the start of the slab
    basis_local(t, p, p, 0.0, v, nullptr);
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j) Kt(i, j) += v[i] * v[j];
}

// Boehm knot insertion: inserts the knots `ins` (one at a time) into the
// knot vector t of degree p and returns the coefficients of every original
// basis function in the refined basis (row i: refined function i).
static std::vector<std::vector<double>> insert_knots(std::vector<double> t, int p, const std::vector<double>& ins) {
    const int Nc = int(t.size()) - p - 1;
    std::vector<std::vector<double>> C(Nc, std::vector<double>(Nc, 0.0));
    for (int i = 0; i < Nc; ++i) C[i][i] = 1.0;
    for (double x : ins) {
        int N = int(t.size()) - p - 1;
        int k = find_span(t, p, x);
        // largest k with t[k] <= x (find_span returns the span containing x)
        while (k + 1 < int(t.size()) && t[k + 1] <= x && k + 1 < N) ++k;
        std::vector<std::vector<double>> Cn(N + 1, std::vector<double>(Nc, 0.0));
        for (int i = 0; i <= N; ++i) {
            if (i <= k - p) {
                Cn[i] = C[i];
            } else if (i >= k + 1) {
                Cn[i] = C[i - 1];
            } else {
                double al = (x - t[i]) / (t[i + p] - t[i]);
                for (int j = 0; j < Nc; ++j) Cn[i][j] = al * C[i][j] + (1.0 - al) * C[i - 1][j];
            }
        }
        C.swap(Cn);
        t.insert(t.begin() + k + 1, x);
    }
    return C;
}

void time_prolongation(int n_el, int p, Mat& Pt) {
    // Coarse slab [0,2] (n_el elements, degree p) represented in the two
    // fine slabs [0,1], [1,2] by Boehm knot insertion: insert every fine
    // knot that is missing, and the slab interface 1 up to multiplicity p+1,
    // which splits the basis into the two fine slab bases.  (The map does
    // not depend on the slab length, so unit slabs are used.)
    std::vector<double> t = open_knots(0.0, 2.0, n_el, p);
    std::vector<double> target;
    for (int i = 0; i <= p; ++i) target.push_back(0.0);
    for (int k = 1; k < n_el; ++k) target.push_back(double(k) / n_el);
    for (int i = 0; i <= p; ++i) target.push_back(1.0);
    for (int k = 1; k < n_el; ++k) target.push_back(1.0 + double(k) / n_el);
    for (int i = 0; i <= p; ++i) target.push_back(2.0);
    // insert target knots not yet present (multiset difference)
    std::vector<double> ins;
    {
        std::vector<double> have = t;
        for (double x : target) {
            auto it = std::find_if(have.begin(), have.end(), [&](double y) { return std::fabs(y - x) < 1e-14; });
            if (it != have.end()) have.erase(it); else ins.push_back(x);
        }
    }
    std::vector<std::vector<double>> C = insert_knots(t, p, ins);
    int Nt = n_el + p;
    Pt = Mat(2 * Nt, Nt);
    for (int i = 0; i < 2 * Nt; ++i)
        for (int j = 0; j < Nt; ++j) Pt(i, j) = C[i][j];
}

void space_prolongation(int n_elem_c, int p, Mat& Px) {
    // Coarse mesh of n_elem_c elements on (0,1) refined by inserting every
    // element midpoint (Boehm); the interior block, since coarse interior
    // functions vanish on the boundary and so have no weight on the first
    // and last fine function
    std::vector<double> ins;
    for (int k = 0; k < n_elem_c; ++k) ins.push_back((2.0 * k + 1.0) / (2.0 * n_elem_c));
    std::vector<std::vector<double>> C = insert_knots(open_knots(0.0, 1.0, n_elem_c, p), p, ins);
    const int nc = n_elem_c + p - 2, nf = 2 * n_elem_c + p - 2;
    Px = Mat(nf, nc);
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nc; ++j) Px(i, j) = C[i + 1][j + 1];
}

void load_time(const Problem& pr, double omega, double phase, std::vector<double>& out) {
    const double pi = 3.14159265358979323846;
    int p = pr.degree, Nt = pr.Nt(), S = pr.n_slabs;
    double tau = pr.tau(), sig = pr.sigma();
    std::vector<double> gx, gw;
    gauss_legendre(p + 3, gx, gw);
    out.assign(size_t(S) * Nt, 0.0);
    std::vector<double> t = open_knots(0.0, tau, pr.n_elem_t, p);
    double v[kMaxDeg + 1], d[kMaxDeg + 1];
    for (int s = 0; s < S; ++s) {
        double t0 = s * tau;
        for (int e = 0; e < pr.n_elem_t; ++e) {
            int span = e + p;
            double a = t[span], b = t[span + 1];
            for (int q = 0; q < p + 3; ++q) {
                double x = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
                double w = 0.5 * (b - a) * gw[q];
                basis_local(t, p, span, x, v, d);
                double f = std::cos(omega * pi * (t0 + x) + phase);
                for (int i = 0; i <= p; ++i) out[size_t(s) * Nt + e + i] += w * f * (v[i] + sig * d[i]);
            }
        }
    }
}

void load_space(const Problem& pr, int k, std::vector<double>& out) {
    const double pi = 3.14159265358979323846;
    int p = pr.degree, ne = pr.n_elem;
    std::vector<double> t = open_knots(0.0, 1.0, ne, p);
    std::vector<double> gx, gw;
    gauss_legendre(p + 3, gx, gw);
    std::vector<double> full(ne + p, 0.0);
    double v[kMaxDeg + 1];
    for (int e = 0; e < ne; ++e) {
        int span = e + p;
        double a = t[span], b = t[span + 1];
        for (int q = 0; q < p + 3; ++q) {
            double x = 0.5 * (b - a) * gx[q] + 0.5 * (a + b);
            double w = 0.5 * (b - a) * gw[q];
            basis_local(t, p, span, x, v, nullptr);
            double f = std::sin(k * pi * x);
            for (int i = 0; i <= p; ++i) full[e + i] += w * f * v[i];
        }
    }
    out.assign(full.begin() + 1, full.end() - 1);
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
int space_transition(const Problem& p) {
    if (!(p.space_ratio > 0.0)) return 0;
    long S = p.n_slabs;
    double tau = p.tau();
    const double ne = p.n_elem;            // h = 1 / n_elem: tau / h^2 = tau n_elem^2
    int lvl = 0;
    while (S > p.coarse_slabs && S % 2 == 0) {
        if (p.n_elem % 2 == 0 && p.n_elem / 2 >= 2 && tau * ne * ne >= p.space_ratio) return lvl + 1;
        S /= 2;
        tau *= 2.0;
        ++lvl;
    }
    return 0;
}

std::string validate(const Problem& p) {
    std::ostringstream os;
    if (p.dim != 2 && p.dim != 3) os << "dim must be 2 or 3; ";
    if (p.degree < 1 || p.degree > kMaxDeg) os << "degree must be in 1.." << kMaxDeg << "; ";
    if (p.n_elem < 2) os << "n_elem must be >= 2; ";
    if (p.n_elem + p.degree - 2 > 1024) os << "n_elem + degree - 2 must be <= 1024; ";
    if (p.n_slabs < 1) os << "n_slabs must be >= 1; ";
    if (p.n_elem_t < 1) os << "n_elem_t must be >= 1; ";
    if (p.n_elem_t + p.degree > kMaxNt) os << "N_t = n_elem_t + degree must be <= " << kMaxNt << "; ";
    if (!(p.T > 0)) os << "T must be > 0; ";
    if (!(p.theta >= 0)) os << "theta must be >= 0; ";
    if (!(p.omega > 0 && p.omega <= 1)) os << "omega must be in (0,1]; ";
    if (p.nu_pre < 0 || p.nu_post < 0 || p.nu_pre + p.nu_post < 1) os << "nu_pre, nu_post >= 0 with a positive sum; ";
    if (p.prec < 0 || p.prec > 2) os << "transform_prec must be 0, 1 or 2; ";
    if (p.coarse_slabs < 1) os << "coarse_slabs must be >= 1; ";
    if (p.temporal < 0 || p.temporal > 2) os << "temporal_form must be 0, 1 or 2; ";
    if (!(p.space_ratio >= 0.0) || !std::isfinite(p.space_ratio)) os << "space_ratio must be finite and >= 0; ";
    if (p.space_ratio > 0.0 && p.basis != 0)
        os << "coarsening in space runs in the B-spline coefficient iteration (iterate_basis 0); ";
    if (p.minres_iters < 0 || p.minres_iters > 200) os << "minres_iters must be in 0..200; ";
    if (p.minres_iters > 0 && p.basis != 0)
        os << "the MinRes slab inverse runs in the B-spline coefficient iteration (iterate_basis 0); ";
    if (p.minres_iters > 0 && p.temporal == 1)
        os << "the MinRes slab inverse needs the temporal eigen form (temporal_form 0 or 2); ";
    if (os.str().empty() && p.n_elem + p.degree - 2 >= 1) {
        double len = double(p.n_slabs) * (p.n_elem_t + p.degree);
        for (int a = 0; a < p.dim; ++a) len *= (p.n_elem + p.degree - 2);
        if (len > 4.0e9) os << "vector length exceeds 4e9; ";
    }
    return os.str();
}

// Eigen form K_t V = M_t V Z (Section 3.3, real 2x2 blocks for conjugate
// pairs), W = (M_t V)^{-1}; the Re(lambda) > 0 guard of Section 3.2.
static int eigen_form(TemporalLevel& L, std::string& err) {
    int Nt = L.Kt.r;
    // M_t positivity: every eigenvalue of M_t must have positive real part
    // (the '*' entries of Table 2 violate this).
    std::vector<cd> lm;
    std::vector<std::vector<cd>> vm;
    if (!nonsym_eigen(L.Mt, lm, vm)) { err = "eigenvalues of M_t did not converge"; return -5; }
    for (auto& z : lm)
        if (z.real() <= 0) { err = "M_t is not positive (reduce theta)"; return -4; }
    Mat Minv;
    if (!lu_inverse(L.Mt, Minv)) { err = "M_t singular"; return -4; }
    Mat C(Nt, Nt);
    for (int i = 0; i < Nt; ++i)
        for (int j = 0; j < Nt; ++j) {
            double s = 0.0;
            for (int k = 0; k < Nt; ++k) s += Minv(i, k) * L.Kt(k, j);
            C(i, j) = s;
        }
    std::vector<cd> lam;
    std::vector<std::vector<cd>> vec;
    if (!nonsym_eigen(C, lam, vec)) { err = "temporal eigen decomposition did not converge"; return -5; }
    double scale = 0.0;
    for (auto& z : lam) scale = std::max(scale, std::abs(z));
    std::vector<int> used(Nt, 0);
    L.V = Mat(Nt, Nt);
    L.re.assign(Nt, 0.0);
    L.im.assign(Nt, 0.0);
    L.kind.assign(Nt, 0);
    // order: by real part, pairs kept adjacent
    std::vector<int> order(Nt);
    for (int i = 0; i < Nt; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
        return lam[a].imag() > lam[b].imag();
    });
    int col = 0;
    for (int oi = 0; oi < Nt; ++oi) {
        int i = order[oi];
        if (used[i]) continue;
        if (lam[i].real() <= 0) {
            std::ostringstream os;
            os << "temporal eigenvalue with Re <= 0 (" << lam[i].real() << "), reduce theta";
            err = os.str();
            return -4;
        }
        if (std::fabs(lam[i].imag()) <= 1e-9 * scale) {
            used[i] = 1;
            // real eigenvector: rotate the complex vector to be real
            std::vector<cd>& x = vec[i];
            int imax = 0;
            for (int r = 1; r < Nt; ++r) if (std::abs(x[r]) > std::abs(x[imax])) imax = r;
            cd ph = std::conj(x[imax]) / std::abs(x[imax]);
            double nn = 0.0;
            for (int r = 0; r < Nt; ++r) { L.V(r, col) = (x[r] * ph).real(); nn += L.V(r, col) * L.V(r, col); }
            nn = std::sqrt(nn);
            for (int r = 0; r < Nt; ++r) L.V(r, col) /= nn;
            L.re[col] = lam[i].real();
            L.im[col] = 0.0;
            L.kind[col] = 0;
            col += 1;
        } else {
            // find the conjugate partner
            int j = -1;
            double best = INFINITY;
            for (int k = 0; k < Nt; ++k) {
                if (k == i || used[k]) continue;
                double dd = std::abs(lam[k] - std::conj(lam[i]));
                if (dd < best) { best = dd; j = k; }
            }
            if (j < 0 || best > 1e-6 * scale || col + 2 > Nt) {
                err = "unpaired complex temporal eigenvalue";
                return -5;
            }
            used[i] = used[j] = 1;
            int ip = lam[i].imag() > 0 ? i : j;       // a + ib with b > 0
            // canonical eigenvector: unit 2-norm, its largest-modulus entry
            // real and positive (the first of equal ones), so that the 2x2
            // spatial block systems of the pair depend on the pencil alone
            std::vector<cd> x = vec[ip];
            {
                int imax = 0;
                for (int r = 1; r < Nt; ++r) if (std::abs(x[r]) > std::abs(x[imax])) imax = r;
                const cd ph = std::conj(x[imax]) / std::abs(x[imax]);
                double nn = 0.0;
                for (int r = 0; r < Nt; ++r) {
                    x[r] *= ph;
                    nn += std::norm(x[r]);
                }
                nn = std::sqrt(nn);
                for (int r = 0; r < Nt; ++r) x[r] /= nn;
            }
            double a = lam[ip].real(), b = lam[ip].imag();
            // K (xr + i xi) = (a + ib) M (xr + i xi)  =>  K V = M V [[a, b], [-b, a]]
            for (int r = 0; r < Nt; ++r) {
                L.V(r, col) = x[r].real();
                L.V(r, col + 1) = x[r].imag();
            }
            L.re[col] = L.re[col + 1] = a;
            L.im[col] = b;
            L.im[col + 1] = -b;
            L.kind[col] = 1;
            L.kind[col + 1] = 2;
            col += 2;
        }
    }
    if (col != Nt) { err = "temporal eigen decomposition incomplete"; return -5; }
    L.condV = cond2(L.V);
    Mat MV(Nt, Nt);
    for (int i = 0; i < Nt; ++i)
        for (int j = 0; j < Nt; ++j) {
            double s = 0.0;
            for (int k = 0; k < Nt; ++k) s += L.Mt(i, k) * L.V(k, j);
            MV(i, j) = s;
        }
    if (!lu_inverse(MV, L.W)) { err = "M_t V singular"; return -5; }
    return 0;
}

// Real Schur form of M_t^{-1} K_t = Q R Q^T (Q orthogonal, R quasi upper
// triangular), so that A_mu = K_t + mu M_t = M_t Q (R + mu I) Q^T and
// A_mu^{-1} = Q (R + mu I)^{-1} Q^T M_t^{-1}: V = Q, W = Q^T M_t^{-1} and a
// block back substitution per spatial mode instead of the diagonal divide.
// Orthogonal temporal transforms whatever cond(V) (the Schur alternative of
// Section 3.3).
static int schur_form(TemporalLevel& L, std::string& err) {
    const int Nt = L.Kt.r;
    Mat Minv;
    if (!lu_inverse(L.Mt, Minv)) { err = "M_t singular"; return -4; }
    Mat C(Nt, Nt);
    for (int i = 0; i < Nt; ++i)
        for (int j = 0; j < Nt; ++j) {
            double v = 0.0;
            for (int k = 0; k < Nt; ++k) v += Minv(i, k) * L.Kt(k, j);
            C(i, j) = v;
        }
    Mat T, Q;
    if (!real_schur(C, T, Q)) { err = "real Schur form did not converge"; return -5; }
    L.schur = true;
    L.R = T;
    L.V = Q;
    L.W = Mat(Nt, Nt);
    for (int i = 0; i < Nt; ++i)
        for (int j = 0; j < Nt; ++j) {
            double v = 0.0;
            for (int k = 0; k < Nt; ++k) v += Q(k, i) * Minv(k, j);
            L.W(i, j) = v;
        }
    L.kind.assign(Nt, 0);
    L.re.assign(Nt, 0.0);
    L.im.assign(Nt, 0.0);
    for (int k = 0; k < Nt;) {
        if (k + 1 < Nt && T(k + 1, k) != 0.0) {
            // eigenvalues of the 2x2 block
            const double a = T(k, k), b = T(k, k + 1), c = T(k + 1, k), d = T(k + 1, k + 1);
            const double tr = 0.5 * (a + d), det = a * d - b * c, disc = tr * tr - det;
            if (disc < 0) {
                L.re[k] = L.re[k + 1] = tr;
                L.im[k] = std::sqrt(-disc);
                L.im[k + 1] = -L.im[k];
            } else {
                L.re[k] = tr + std::sqrt(disc);
                L.re[k + 1] = tr - std::sqrt(disc);
            }
            L.kind[k] = 1;
            L.kind[k + 1] = 2;
            k += 2;
        } else {
            L.re[k] = T(k, k);
            k += 1;
        }
    }
    for (int k = 0; k < Nt; ++k)
        if (L.re[k] <= 0) { err = "temporal eigenvalue with Re <= 0, reduce theta"; return -4; }
    return 0;
}

// temporal: 0 diagonalisation (STH_ECOND above cond(V) = 1e8), 1 real
// Schur, 2 diagonalisation unless cond(V) > 1e6, then real Schur
static int temporal_decomposition(TemporalLevel& L, int temporal, std::string& err) {
    int st = eigen_form(L, err);
    if (st == -4) return st;                       // positivity guard, whatever the form
    const bool use_schur = temporal == 1 || (temporal == 2 && (st != 0 || !(L.condV <= 1e6)));
    if (use_schur) {
        const double condV = st == 0 ? L.condV : INFINITY;
        err.clear();
        st = schur_form(L, err);
        L.condV = condV;
        return st;
    }
    if (st) return st;
    if (!(L.condV <= 1e8)) {
        std::ostringstream os;
        os << "cond(V) = " << L.condV << " too large for the diagonalisation path";
        err = os.str();
        return -5;
    }
    return 0;
}

// Eigenpairs of the symmetric pencil (K, M), M positive definite:
// M = L L^T, L^{-1} K L^{-T} = Q diag(mu) Q^T, U = L^{-T} Q (U^T M U = I),
// mu ascending.
static bool pencil_eigen(const Mat& K, const Mat& M, std::vector<double>& mu, Mat& U) {
    Mat Lc;
    if (!cholesky(M, Lc)) return false;
    const int n = M.r;
    Mat Linv(n, n);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= Lc(i, k) * Linv(k, j);
            Linv(i, j) = v / Lc(i, i);
        }
    }
    Mat T1(n, n), C(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = 0.0;
            for (int k = 0; k <= i; ++k) v += Linv(i, k) * K(k, j);
            T1(i, j) = v;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = 0.0;
            for (int k = 0; k <= j; ++k) v += T1(i, k) * Linv(j, k);
            C(i, j) = v;
        }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) C(i, j) = C(j, i) = 0.5 * (C(i, j) + C(j, i));
    Mat Q;
    sym_eigen(C, mu, Q);
    U = Mat(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = 0.0;
            for (int k = i; k < n; ++k) v += Linv(k, i) * Q(k, j);
            U(i, j) = v;
        }
    return true;
}

// A(i, j) = A(n-1-i, n-1-j) to rounding
static bool reflection_symmetric(const Mat& A) {
    const int n = A.r;
    double amax = 0.0, d = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            amax = std::max(amax, std::fabs(A(i, j)));
            d = std::max(d, std::fabs(A(i, j) - A(n - 1 - i, n - 1 - j)));
        }
    return d <= 1e-12 * amax;
}

int build_setup(const Problem& p, Setup& s, std::string& err) {
    err = validate(p);
    if (!err.empty()) return -1;
    s.prob = p;
    s.n = p.n();
    s.Nt = p.Nt();
    space_matrices(p.n_elem, p.degree, s.M1, s.K1);
    const int n = s.n;
    const int h = n / 2;
    if (n % 2 == 0 && reflection_symmetric(s.M1) && reflection_symmetric(s.K1)) {
        // The reflection J (i -> n - 1 - i) commutes with M1 and K1, so the
        // eigenvectors split into even ones, v = [w; J w], and odd ones,
        // v = [w; -J w], where w solves the half pencil (K11 +- K12 J,
        // M11 +- M12 J) of order n / 2.  With w^T (M11 +- M12 J) w = 1,
        // v / sqrt 2 is M1-orthonormal.
        Mat U(n, n);
        s.mu.assign(n, 0.0);
        for (int sg = 0; sg < 2; ++sg) {
            const double sign = sg == 0 ? 1.0 : -1.0;
            Mat Kh(h, h), Mh(h, h);
            for (int i = 0; i < h; ++i)
                for (int j = 0; j < h; ++j) {
                    Kh(i, j) = s.K1(i, j) + sign * s.K1(i, n - 1 - j);
                    Mh(i, j) = s.M1(i, j) + sign * s.M1(i, n - 1 - j);
                }
            std::vector<double> mh;
            Mat Uh;
            if (!pencil_eigen(Kh, Mh, mh, Uh)) {
                err = "half mass matrix not positive definite";
                return -5;
            }
            if (p.basis == 1) {
                // the eigenvalues of M1 are those of its two half matrices
                std::vector<double> ev;
                Mat Qm;
                sym_eigen(Mh, ev, Qm);
                const double lo = *std::min_element(ev.begin(), ev.end());
                const double hi = *std::max_element(ev.begin(), ev.end());
                s.m1_min = sg == 0 ? lo : std::min(s.m1_min, lo);
                s.m1_max = sg == 0 ? hi : std::max(s.m1_max, hi);
            }
            const double r2 = std::sqrt(0.5);
            for (int j = 0; j < h; ++j) {
                s.mu[sg * h + j] = mh[j];
                for (int i = 0; i < h; ++i) {
                    U(i, sg * h + j) = r2 * Uh(i, j);
                    U(n - 1 - i, sg * h + j) = sign * r2 * Uh(i, j);
                }
            }
        }
        s.U = U;
        s.half = h;
    } else {
        if (!pencil_eigen(s.K1, s.M1, s.mu, s.U)) {
            err = "M1 not positive definite";
            return -5;
        }
        s.half = 0;
    }
    if (p.basis == 1 && s.half == 0) {
        // C = M1 U satisfies C C^T = M1 (U U^T = M1^{-1}), so the squared
        // singular values of C are the eigenvalues of M1
        std::vector<double> ev;
        Mat Qm;
        sym_eigen(s.M1, ev, Qm);
        s.m1_min = *std::min_element(ev.begin(), ev.end());
        s.m1_max = *std::max_element(ev.begin(), ev.end());
    }
    // temporal levels
    s.levels.clear();
    int S = p.n_slabs;
    double tau = p.tau();
    Mat Pt;
    time_prolongation(p.n_elem_t, p.degree, Pt);
    while (true) {
        TemporalLevel L;
        L.S = S;
        L.tau = tau;
        time_matrices(tau, p.n_elem_t, p.degree, p.sigma(), L.Kt, L.Mt);
        int st = temporal_decomposition(L, p.temporal, err);
        if (st != 0) {
            std::ostringstream os;
            os << "level " << s.levels.size() << ": " << err;
            err = os.str();
            return st;
        }
        bool coarsen = (S > p.coarse_slabs && S % 2 == 0) &&
                       (p.level_cap <= 0 || (int)s.levels.size() + 1 < p.level_cap);
        if (coarsen) L.Pt = Pt;
        s.levels.push_back(L);
        if (!coarsen) break;
        S /= 2;
        tau *= 2;
    }
    return 0;
}

// Lower bound of the B-spline norm of an eigenbasis vector, per mode: with
// G = C^T C = D + E (D its diagonal) and x^T (G (x) G - D (x) D) x bounded by
// the absolute row sums of G (x) G - D (x) D (symmetric), which are
// prod a - prod d for the mode (a the absolute row sums of G).
std::vector<double> residual_mode_weights(const Setup& s) {
    const int n = s.n;
    Mat C(n, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double c = 0.0;
            for (int k = 0; k < n; ++k) c += s.M1(i, k) * s.U(k, j);
            C(i, j) = c;
        }
    std::vector<double> w((size_t)2 * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double g = 0.0;
            for (int k = 0; k < n; ++k) g += C(k, i) * C(k, j);
            if (i == j) w[2 * i] = g;
            w[2 * i + 1] += std::fabs(g);
        }
    return w;
}

}  // namespace sth
