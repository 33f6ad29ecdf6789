// Host-side setup: 1D reference element, fast-diagonalisation data, error
// reporting.
//
// 1D element: Lagrange polynomials on the p+1 Gauss-Lobatto-Legendre nodes of
// [0,1] integrated by the (p+1)-point Gauss-Legendre rule, which is exact for
// the 1D mass (degree 2p) and stiffness (degree 2p-2) integrands.
//
// Fast diagonalisation (Lynch, Rice & Thomas 1964).  On a tensor-product
// patch of 2x2x2 box cells the patch operator is a Kronecker sum
//   A_P = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz
// of 1D matrices assembled over the two cells of each direction and
// restricted to the 2p-1 interior nodes.  With the 1D generalised
// eigenproblems K S = M S diag(lambda), S^T M S = I, the inverse is
//   A_P^{-1} = (Sx (x) Sy (x) Sz) diag(1 / (lx + ly + lz)) (Sx (x) Sy (x) Sz)^T.
// Each 1D problem is reduced to a symmetric one by the Cholesky factor of M
// and solved by cyclic Jacobi rotations in FP64.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdint>
#include <unordered_map>
#include <mutex>
#include <string>
#include <vector>

#include "fem_internal.h"
#include "launch.h"
#include "host_api.h"

namespace fem {

static thread_local std::string g_last_error;

fem_status set_error(fem_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

fem_status hip_error(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(FEM_EHIP, m);
}

// ------------------------------------------------------------ 1D rules
static void legendre(int n, double x, double* P, double* dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *P = p1;
    *dP = n * (x * p1 - p0) / (x * x - 1.0);   // interior points only
}

// GLL nodes on [0,1].
std::vector<double> host_gll_nodes(int p) {
    std::vector<double> s(p + 1);
    s[0] = -1.0;
    s[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double x = -std::cos(M_PI * k / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, x, &P, &dP);
            double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        s[k] = x;
    }
    std::sort(s.begin(), s.end());
    std::vector<double> out(p + 1);
    for (int i = 0; i <= p; ++i) out[i] = 0.5 * (s[i] + 1.0);
    out[0] = 0.0;
    out[p] = 1.0;
    return out;
}

// Gauss-Legendre rule with nq points on [0,1].
void host_gauss(int nq, std::vector<double>& x, std::vector<double>& w) {
    x.assign(nq, 0.0);
    w.assign(nq, 0.0);
    for (int k = 0; k < nq; ++k) {
        double t = -std::cos(M_PI * (k + 0.75) / (nq + 0.5));
        double P = 0, dP = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(nq, t, &P, &dP);
            double dt = P / dP;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        legendre(nq, t, &P, &dP);
        x[k] = 0.5 * (t + 1.0);
        w[k] = 1.0 / ((1.0 - t * t) * dP * dP);   // 2/((1-t^2)P'^2) halved for [0,1]
    }
}

void host_ref_matrices(int p, double* M, double* K) {
    const int n1 = p + 1;
    std::vector<double> xi = host_gll_nodes(p), xq, wq;
    host_gauss(n1, xq, wq);
    std::vector<double> V(n1 * n1), D(n1 * n1);   // [q][a]
    for (int q = 0; q < n1; ++q) {
        for (int a = 0; a < n1; ++a) {
            double v = 1.0, d = 0.0;
            for (int b = 0; b < n1; ++b)
                if (b != a) v *= (xq[q] - xi[b]) / (xi[a] - xi[b]);
            for (int m = 0; m < n1; ++m) {
                if (m == a) continue;
                double t = 1.0 / (xi[a] - xi[m]);
                for (int b = 0; b < n1; ++b)
                    if (b != a && b != m) t *= (xq[q] - xi[b]) / (xi[a] - xi[b]);
                d += t;
            }
            V[q * n1 + a] = v;
            D[q * n1 + a] = d;
        }
    }
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) {
            double sm = 0, sk = 0;
            for (int q = 0; q < n1; ++q) {
                sm += wq[q] * V[q * n1 + a] * V[q * n1 + b];
                sk += wq[q] * D[q * n1 + a] * D[q * n1 + b];
            }
            M[a * n1 + b] = sm;
            K[a * n1 + b] = sk;
        }
}

static std::once_flag g_ref_once;
static double g_ref_M[kMaxP + 1][(kMaxP + 1) * (kMaxP + 1)];
static double g_ref_K[kMaxP + 1][(kMaxP + 1) * (kMaxP + 1)];

static void init_refs() {
    for (int p = 1; p <= kMaxP; ++p) host_ref_matrices(p, g_ref_M[p], g_ref_K[p]);
}
const double* ref_mass(int p) {
    std::call_once(g_ref_once, init_refs);
    return g_ref_M[p];
}
const double* ref_stiff(int p) {
    std::call_once(g_ref_once, init_refs);
    return g_ref_K[p];
}

// ---------------------------------------------------- 1D fast diagonalisation
// Symmetric eigen-decomposition by cyclic Jacobi: A (n x n, row-major) is
// destroyed; Q receives the eigenvectors as columns, lam the eigenvalues.
static void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& lam) {
    Q.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    double fro = 0;
    for (double v : A) fro += v * v;
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (std::sqrt(off) <= 1e-17 * fro) break;
        for (int pi = 0; pi < n; ++pi)
            for (int qi = pi + 1; qi < n; ++qi) {
                double apq = A[pi * n + qi];
                if (apq == 0.0) continue;
                double app = A[pi * n + pi], aqq = A[qi * n + qi];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {          // A <- A J
                    double akp = A[k * n + pi], akq = A[k * n + qi];
                    A[k * n + pi] = c * akp - s * akq;
                    A[k * n + qi] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          // A <- J^T A
                    double apk = A[pi * n + k], aqk = A[qi * n + k];
                    A[pi * n + k] = c * apk - s * aqk;
                    A[qi * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {          // Q <- Q J
                    double qkp = Q[k * n + pi], qkq = Q[k * n + qi];
                    Q[k * n + pi] = c * qkp - s * qkq;
                    Q[k * n + qi] = s * qkp + c * qkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

// 1D patch matrices of two cells (widths h0, h1) on the 2p-1 interior nodes.
void host_patch_1d(int p, double h0, double h1, std::vector<double>& M, std::vector<double>& K) {
    const int n1 = p + 1, nP = 2 * p - 1;
    const double* Mr = ref_mass(p);
    const double* Kr = ref_stiff(p);
    M.assign(nP * nP, 0.0);
    K.assign(nP * nP, 0.0);
    for (int cell = 0; cell < 2; ++cell) {
        const double h = cell == 0 ? h0 : h1;
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n1; ++b) {
                int I = cell * p + a - 1, J = cell * p + b - 1;    // interior index
                if (I < 0 || I >= nP || J < 0 || J >= nP) continue;
                M[I * nP + J] += h * Mr[a * n1 + b];
                K[I * nP + J] += Kr[a * n1 + b] / h;
            }
    }
}

static int host_fd_1d_compute(int p, double h0, double h1, double* S, double* lam);
int host_gen_eig(int n, const std::vector<double>& M, const std::vector<double>& K, double* S, double* lam);

// The 1D data depend only on (p, h0, h1); uniform meshes and repeated
// requests reuse them, so results are memoised (bounded, process-wide).
int host_fd_1d(int p, double h0, double h1, double* S, double* lam) {
    struct Key {
        int p;
        uint64_t a, b;
        bool operator==(const Key& o) const { return p == o.p && a == o.a && b == o.b; }
    };
    struct KeyHash {
        size_t operator()(const Key& k) const {
            return std::hash<uint64_t>()(k.a * 0x9E3779B97F4A7C15ull ^ (k.b + (uint64_t)k.p * 0x632BE59BD9B4E019ull));
        }
    };
    static std::mutex mu;
    static std::unordered_map<Key, std::vector<double>, KeyHash> cache;
    const int n = 2 * p - 1;
    Key key{p, 0, 0};
    std::memcpy(&key.a, &h0, 8);
    std::memcpy(&key.b, &h1, 8);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            std::memcpy(S, it->second.data(), sizeof(double) * n * n);
            std::memcpy(lam, it->second.data() + n * n, sizeof(double) * n);
            return 0;
        }
    }
    const int rc = host_fd_1d_compute(p, h0, h1, S, lam);
    if (rc != 0) return rc;
    std::vector<double> v(S, S + n * n);
    v.insert(v.end(), lam, lam + n);
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() >= 16384) cache.clear();
    cache.emplace(key, std::move(v));
    return 0;
}

static int host_fd_1d_compute(int p, double h0, double h1, double* S, double* lam) {
    std::vector<double> M, K;
    host_patch_1d(p, h0, h1, M, K);
    return host_gen_eig(2 * p - 1, M, K, S, lam);
}

// 1D Q1 matrices on the interior vertices of a 1D mesh of n cells (widths h)
// with homogeneous Dirichlet ends: tridiagonal stiffness (1/h per cell) and
// consistent mass (h/3 on the diagonal per cell, h/6 off it).
void host_q1_1d(int n, const double* h, std::vector<double>& M, std::vector<double>& K) {
    const int m = n - 1;
    M.assign((size_t)m * m, 0.0);
    K.assign((size_t)m * m, 0.0);
    for (int c = 0; c < n; ++c) {          // cell c joins vertices c and c+1 (interior index c-1, c)
        const int i0 = c - 1, i1 = c;
        const double kh = 1.0 / h[c], mh = h[c];
        if (i0 >= 0) {
            K[i0 * m + i0] += kh;
            M[i0 * m + i0] += mh / 3.0;
        }
        if (i1 < m) {
            K[i1 * m + i1] += kh;
            M[i1 * m + i1] += mh / 3.0;
        }
        if (i0 >= 0 && i1 < m) {
            K[i0 * m + i1] -= kh;
            K[i1 * m + i0] -= kh;
            M[i0 * m + i1] += mh / 6.0;
            M[i1 * m + i0] += mh / 6.0;
        }
    }
}

int host_coarse_1d(int n, const double* h, double* S, double* lam) {
    if (n < 2) return 0;
    std::vector<double> M, K;
    host_q1_1d(n, h, M, K);
    return host_gen_eig(n - 1, M, K, S, lam);
}

// Generalised symmetric eigenproblem K S = M S diag(lam), S^T M S = I, M SPD
// (n x n, row-major): Cholesky M = L L^T, cyclic Jacobi on L^{-1} K L^{-T},
// S = L^{-T} Q; ascending eigenvalues, each eigenvector's largest-magnitude
// entry positive.
int host_gen_eig(int n, const std::vector<double>& M, const std::vector<double>& K, double* S, double* lam) {
    // Cholesky M = L L^T
    std::vector<double> L(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = M[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0)) return -1;
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = M[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    // Y = L^{-1} K (forward substitution per column), C = L^{-1} Y^T
    auto fwd = [&](const std::vector<double>& B, std::vector<double>& X) {
        X.assign(n * n, 0.0);
        for (int col = 0; col < n; ++col)
            for (int i = 0; i < n; ++i) {
                double v = B[i * n + col];
                for (int k = 0; k < i; ++k) v -= L[i * n + k] * X[k * n + col];
                X[i * n + col] = v / L[i * n + i];
            }
    };
    std::vector<double> Y, Yt(n * n), C;
    fwd(K, Y);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Yt[i * n + j] = Y[j * n + i];
    fwd(Yt, C);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double a = 0.5 * (C[i * n + j] + C[j * n + i]);
            C[i * n + j] = C[j * n + i] = a;
        }
    std::vector<double> Q, ev;
    jacobi_eigen(n, C, Q, ev);
    // S = L^{-T} Q (back substitution per column)
    std::vector<double> Sm(n * n, 0.0);
    for (int col = 0; col < n; ++col)
        for (int i = n - 1; i >= 0; --i) {
            double v = Q[i * n + col];
            for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * Sm[k * n + col];
            Sm[i * n + col] = v / L[i * n + i];
        }
    // ascending eigenvalues; eigenvector sign: largest-magnitude entry positive
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return ev[a] < ev[b]; });
    for (int j = 0; j < n; ++j) {
        int src = ord[j];
        int imax = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(Sm[i * n + src]) > std::fabs(Sm[imax * n + src])) imax = i;
        double sg = Sm[imax * n + src] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < n; ++i) S[i * n + j] = sg * Sm[i * n + src];
        lam[j] = ev[src];
        if (!(lam[j] > 0)) return -2;
    }
    return 0;
}

}  // namespace fem

using namespace fem;

namespace fem {
extern std::atomic<int> g_pi_fused;
extern std::atomic<int> g_combine_per_cell;
extern std::atomic<int> g_restrict_from_cells;
extern std::atomic<int> g_pi_slab_mb;
extern std::atomic<int> g_apply_planes_p7;
}  // namespace fem

extern "C" fem_status fem_set_option(int option, int value) {
    switch (option) {
        case FEM_OPT_PI_FUSED:
            if (value < -1 || value > 4) return set_error(FEM_EINVAL, "fem_set_option: FEM_OPT_PI_FUSED is -1..4");
            fem::g_pi_fused = value;
            return FEM_OK;
        case FEM_OPT_COMBINE_PER_CELL:
            if (value < 0 || value > 2) return set_error(FEM_EINVAL, "fem_set_option: FEM_OPT_COMBINE_PER_CELL is 0..2");
            fem::g_combine_per_cell = value;
            return FEM_OK;
        case FEM_OPT_RESTRICT_FROM_CELLS: fem::g_restrict_from_cells = value ? 1 : 0; return FEM_OK;
        case FEM_OPT_PI_SLAB_MB:
            if (value < 0) return set_error(FEM_EINVAL, "fem_set_option: FEM_OPT_PI_SLAB_MB >= 0");
            fem::g_pi_slab_mb = value;
            return FEM_OK;
        case FEM_OPT_APPLY_PLANES_P7: fem::g_apply_planes_p7 = value ? 1 : 0; return FEM_OK;
        default: return set_error(FEM_EINVAL, "fem_set_option: unknown option");
    }
}

extern "C" const char* fem_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* fem_version(void) { return "fem-mi355x 0.1 (gfx950)"; }

extern "C" fem_status fem_host_1d_matrices(int p, double* mass, double* stiff) {
    if (p < 1 || p > kMaxP || !mass || !stiff) return set_error(FEM_EINVAL, "fem_host_1d_matrices: p in 1..7");
    std::memcpy(mass, ref_mass(p), sizeof(double) * (p + 1) * (p + 1));
    std::memcpy(stiff, ref_stiff(p), sizeof(double) * (p + 1) * (p + 1));
    return FEM_OK;
}

extern "C" fem_status fem_host_gll_nodes(int p, double* nodes) {
    if (p < 1 || p > kMaxP || !nodes) return set_error(FEM_EINVAL, "fem_host_gll_nodes: p in 1..7");
    std::vector<double> x = host_gll_nodes(p);
    std::memcpy(nodes, x.data(), sizeof(double) * (p + 1));
    return FEM_OK;
}

extern "C" fem_status fem_host_fd_1d(int p, double h0, double h1, double* S, double* lambda) {
    if (p < 1 || p > kMaxP || !S || !lambda || !(h0 > 0) || !(h1 > 0))
        return set_error(FEM_EINVAL, "fem_host_fd_1d: p in 1..7, positive widths");
    if (host_fd_1d(p, h0, h1, S, lambda) != 0)
        return set_error(FEM_EINVAL, "fem_host_fd_1d: 1D patch matrices not positive definite");
    return FEM_OK;
}
