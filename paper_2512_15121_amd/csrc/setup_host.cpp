// Host-side setup of the GIAMG hierarchy: fine assembly, p-transfers,
// smoothed aggregation, transposes and the coarsest dense inverse.
//
// Paper passages: problem A x = b (Section 2); element dof map l2g and the
// tensor dof ordering (Section 2.1.1 "Required geometric information",
// appendix); Algorithms 2-4 (kept dofs, sorted collection, next-level map);
// Algorithm 7 (prolongation, nodal-interpolation variant); Section 2.5
// (MIS aggregation, tentative prolongation, SPAI smoothing).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "internal.h"

namespace giamg {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& fn) {
    if (n <= 0) return;
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int64_t nthreads = std::min<int64_t>(hw, std::max<int64_t>(1, n / std::max<int64_t>(1, grain)));
    if (nthreads <= 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> pool;
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int64_t t = 0; t < nthreads; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        pool.emplace_back([&fn, b, e] { fn(b, e); });
    }
    for (auto& th : pool) th.join();
}

// (i+1)-th output of SplitMix64 started from state `seed` (Steele, Lea and
// Flood 2014): state advances by the golden gamma, output is the mixed state.
uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// 1-D bases and quadrature
// ---------------------------------------------------------------------------
// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
static void legendre(int n, double x, double& P, double& dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    // derivative from (x^2 - 1) P_n' = n (x P_n - P_{n-1}); only used off +-1
    dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// Gauss-Lobatto-Legendre points: +-1 and the roots of P_p', found by Newton
// iteration on P_p' with P_p'' from the Legendre equation
// (1 - x^2) P'' = 2 x P' - p (p + 1) P.  Weights 2 / (p (p+1) P_p(x)^2).
void gll_points(int p, std::vector<double>& x, std::vector<double>& w) {
    x.assign(p + 1, 0.0);
    w.assign(p + 1, 0.0);
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double xi = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, xi, P, dP);
            double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
            double step = dP / d2P;
            xi -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        x[i] = xi;
    }
    // symmetric pairs are made exactly symmetric
    for (int i = 0; i <= p / 2; ++i) {
        double m = 0.5 * (x[p - i] - x[i]);
        x[i] = -m;
        x[p - i] = m;
    }
    if (p % 2 == 0) x[p / 2] = 0.0;
    for (int i = 0; i <= p; ++i) {
        double P, dP;
        if (std::fabs(x[i]) == 1.0) {
            P = (x[i] > 0 || p % 2 == 0) ? 1.0 : -1.0;
        } else {
            legendre(p, x[i], P, dP);
        }
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
}

// Gauss-Legendre points (roots of P_m by Newton), weights 2 / ((1-x^2) P_m'^2).
void gauss_points(int m, std::vector<double>& x, std::vector<double>& w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
        double xi = -std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double P = 0, dP = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(m, xi, P, dP);
            double step = P / dP;
            xi -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        legendre(m, xi, P, dP);
        x[i] = xi;
        w[i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
    }
    for (int i = 0; i < m / 2; ++i) {
        double a = 0.5 * (x[m - 1 - i] - x[i]);
        double ww = 0.5 * (w[i] + w[m - 1 - i]);
        x[i] = -a;
        x[m - 1 - i] = a;
        w[i] = w[m - 1 - i] = ww;
    }
    if (m % 2 == 1) x[m / 2] = 0.0;
}

double lagrange_value(const std::vector<double>& nodes, int i, double x) {
    double v = 1.0;
    for (size_t j = 0; j < nodes.size(); ++j)
        if ((int)j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    return v;
}

double lagrange_derivative(const std::vector<double>& nodes, int i, double x) {
    double s = 0.0;
    for (size_t m = 0; m < nodes.size(); ++m) {
        if ((int)m == i) continue;
        double t = 1.0 / (nodes[i] - nodes[m]);
        for (size_t j = 0; j < nodes.size(); ++j)
            if ((int)j != i && j != m) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
        s += t;
    }
    return s;
}

static inline int lidx(int p, int i, int j, int k) { return ((p + 1) * i + j) * (p + 1) + k; }

// 1-D local index of the vertex mode/node that is one at a = -1 (side 0) or
// a = +1 (side 1): nodal GLL ends 0 and p; the modal ordering of the
// appendix numbers the two vertex modes 0 and 1.
static inline int vend(int p, int basis, int side) {
    return side == 0 ? 0 : (basis == GIAMG_BASIS_MODAL ? 1 : p);
}

// ---------------------------------------------------------------------------
// topology
// ---------------------------------------------------------------------------
// A face is identified by its four corner nodes; a face seen by exactly one
// element lies on the boundary and all of its nodes are constrained.
std::vector<uint8_t> boundary_mask(const int32_t* l2g, int64_t n_elem, int p, int64_t n_nodes,
                                   int basis) {
    const int nl = (p + 1) * (p + 1) * (p + 1);
    const int e0 = vend(p, basis, 0), e1 = vend(p, basis, 1);
    struct Face { int32_t c[4]; int64_t elem; int8_t f; };
    std::vector<Face> faces(n_elem * 6);
    auto face_node = [p, e0, e1](int f, int a, int b) {
        int fixed = (f < 3) ? e0 : e1;
        switch (f % 3) {
            case 0: return lidx(p, fixed, a, b);
            case 1: return lidx(p, a, fixed, b);
            default: return lidx(p, a, b, fixed);
        }
    };
    parallel_for(n_elem, 4096, [&](int64_t b, int64_t e) {
        for (int64_t el = b; el < e; ++el) {
            const int32_t* g = l2g + el * nl;
            for (int f = 0; f < 6; ++f) {
                Face F;
                F.c[0] = g[face_node(f, e0, e0)];
                F.c[1] = g[face_node(f, e0, e1)];
                F.c[2] = g[face_node(f, e1, e0)];
                F.c[3] = g[face_node(f, e1, e1)];
                std::sort(F.c, F.c + 4);
                F.elem = el;
                F.f = (int8_t)f;
                faces[el * 6 + f] = F;
            }
        }
    });
    auto key_less = [](const Face& a, const Face& b) {
        return std::lexicographical_compare(a.c, a.c + 4, b.c, b.c + 4);
    };
    std::sort(faces.begin(), faces.end(), key_less);
    std::vector<uint8_t> mask(n_nodes, 0);
    size_t i = 0;
    while (i < faces.size()) {
        size_t j = i + 1;
        while (j < faces.size() && std::equal(faces[i].c, faces[i].c + 4, faces[j].c)) ++j;
        if (j - i == 1) {
            const int32_t* g = l2g + faces[i].elem * nl;
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p; ++b) mask[g[face_node(faces[i].f, a, b)]] = 1;
        }
        i = j;
    }
    return mask;
}

void element_corners(const double* coords, const int32_t* l2g, int64_t n_elem, int p,
                     std::vector<double>& corners, int basis) {
    const int nl = (p + 1) * (p + 1) * (p + 1);
    corners.assign(n_elem * 24, 0.0);
    for (int64_t e = 0; e < n_elem; ++e)
        for (int c = 0; c < 8; ++c) {
            int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
            int32_t g = l2g[e * nl + lidx(p, vend(p, basis, cx), vend(p, basis, cy), vend(p, basis, cz))];
            for (int a = 0; a < 3; ++a) corners[e * 24 + c * 3 + a] = coords[(int64_t)g * 3 + a];
        }
}

// ---------------------------------------------------------------------------
// element matrices by sum factorisation
// ---------------------------------------------------------------------------
namespace {

struct RefTables {
    int p, nq, n1;                      // n1 = p + 1
    std::vector<double> g, wg;          // 1-D Gauss points / weights
    std::vector<double> L, D;           // [n1][nq] basis values / derivatives
};

// Modal 1-D modes of the appendix through Legendre polynomials: for n >= 2
// the bubble (1-a)/2 (1+a)/2 P^{1,1}_{n-2}(a) equals
// (n-1)/(2(2n-1)) (P_{n-2}(a) - P_n(a)) and its derivative is
// -(n-1)/2 P_{n-1}(a) (Legendre's equation); the vertex modes are (1-a)/2
// and (1+a)/2.
static void modal_value_derivative(int p, double x, double* v, double* d) {
    std::vector<double> P(p + 1);
    P[0] = 1.0;
    if (p >= 1) P[1] = x;
    for (int k = 1; k < p; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    v[0] = 0.5 * (1.0 - x);
    d[0] = -0.5;
    if (p >= 1) {
        v[1] = 0.5 * (1.0 + x);
        d[1] = 0.5;
    }
    for (int n = 2; n <= p; ++n) {
        v[n] = (n - 1) / (2.0 * (2 * n - 1)) * (P[n - 2] - P[n]);
        d[n] = -0.5 * (n - 1) * P[n - 1];
    }
}

RefTables make_tables(int p, int basis) {
    RefTables t;
    t.p = p;
    t.nq = p + 2;
    t.n1 = p + 1;
    gauss_points(t.nq, t.g, t.wg);
    t.L.resize(t.n1 * t.nq);
    t.D.resize(t.n1 * t.nq);
    if (basis == GIAMG_BASIS_MODAL) {
        std::vector<double> v(p + 1), d(p + 1);
        for (int q = 0; q < t.nq; ++q) {
            modal_value_derivative(p, t.g[q], v.data(), d.data());
            for (int i = 0; i < t.n1; ++i) {
                t.L[i * t.nq + q] = v[i];
                t.D[i * t.nq + q] = d[i];
            }
        }
        return t;
    }
    std::vector<double> xn, wn;
    gll_points(p, xn, wn);
    for (int i = 0; i < t.n1; ++i)
        for (int q = 0; q < t.nq; ++q) {
            t.L[i * t.nq + q] = lagrange_value(xn, i, t.g[q]);
            t.D[i * t.nq + q] = lagrange_derivative(xn, i, t.g[q]);
        }
    return t;
}

// Jacobian of the trilinear map at reference point xi; returns det J.
inline double trilinear_jacobian(const double* X, const double xi[3], double J[3][3]) {
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) J[a][d] = 0.0;
    for (int c = 0; c < 8; ++c) {
        double s[3] = {((c >> 2) & 1) ? 1.0 : -1.0, ((c >> 1) & 1) ? 1.0 : -1.0,
                       (c & 1) ? 1.0 : -1.0};
        double f[3] = {0.5 * (1 + s[0] * xi[0]), 0.5 * (1 + s[1] * xi[1]), 0.5 * (1 + s[2] * xi[2])};
        double dN[3] = {0.5 * s[0] * f[1] * f[2], 0.5 * s[1] * f[0] * f[2], 0.5 * s[2] * f[0] * f[1]};
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) J[a][d] += X[c * 3 + a] * dN[d];
    }
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Element matrix K_e + lambda M_e, row-major [nl][nl], upper triangle mirrored.
// K_e[a][b] = sum_q sum_{d,d'} G_dd'(q) dphi_a/dxi_d dphi_b/dxi_d' with
// G = w |J| J^-1 J^-T; each tensor term is contracted one direction at a time
// (z, then y, then x).  Returns false on a non-positive Jacobian.
bool element_matrix(const RefTables& t, const double* X, double lambda, double* Ke,
                    std::vector<double>& work) {
    const int nq = t.nq, n1 = t.n1, n2 = n1 * n1, nl = n2 * n1;
    const int Q = nq * nq * nq;
    // geometric factors: G[q][6] (xx,xy,xz,yy,yz,zz) and the mass weight
    work.resize((size_t)Q * 7 + (size_t)nq * nq * n2 + 4 * (size_t)nq * n2 * n2 + (size_t)nq * n2 * n2);
    double* G = work.data();
    double* T1 = G + (size_t)Q * 7;
    double* T2g = T1 + (size_t)nq * nq * n2;             // 4 groups of [nq][n2][n2]
    double* T2 = T2g + 4 * (size_t)nq * n2 * n2;
    for (int qx = 0; qx < nq; ++qx)
        for (int qy = 0; qy < nq; ++qy)
            for (int qz = 0; qz < nq; ++qz) {
                double xi[3] = {t.g[qx], t.g[qy], t.g[qz]};
                double J[3][3];
                double det = trilinear_jacobian(X, xi, J);
                if (!(det > 0.0)) return false;
                // inverse: Ji[d][a] = d xi_d / d x_a
                double Ji[3][3];
                Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                double w = t.wg[qx] * t.wg[qy] * t.wg[qz] * det;
                int q = (qx * nq + qy) * nq + qz;
                double* g = G + (size_t)q * 7;
                int m = 0;
                for (int d = 0; d < 3; ++d)
                    for (int e = d; e < 3; ++e) {
                        double s = 0.0;
                        for (int a = 0; a < 3; ++a) s += Ji[d][a] * Ji[e][a];
                        g[m++] = w * s;
                    }
                g[6] = lambda * w;
            }
    static const int gidx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    std::fill(T2g, T2g + 4 * (size_t)nq * n2 * n2, 0.0);
    // ten tensor terms: (d, d') stiffness pairs and the mass term (d = d' = -1)
    for (int term = 0; term < 10; ++term) {
        int d = term < 9 ? term / 3 : -1;
        int e = term < 9 ? term % 3 : -1;
        int gi = term < 9 ? gidx[d][e] : 6;
        const double* Fz = (d == 2) ? t.D.data() : t.L.data();
        const double* Fzp = (e == 2) ? t.D.data() : t.L.data();
        const double* Fy = (d == 1) ? t.D.data() : t.L.data();
        const double* Fyp = (e == 1) ? t.D.data() : t.L.data();
        // T1[qx][qy][k][k'] = sum_qz Fz[k][qz] Fz'[k'][qz] G(qx,qy,qz)
        for (int qx = 0; qx < nq; ++qx)
            for (int qy = 0; qy < nq; ++qy) {
                double* out = T1 + ((size_t)qx * nq + qy) * n2;
                for (int k = 0; k < n1; ++k)
                    for (int kp = 0; kp < n1; ++kp) {
                        double s = 0.0;
                        for (int qz = 0; qz < nq; ++qz)
                            s += Fz[k * nq + qz] * Fzp[kp * nq + qz] *
                                 G[(size_t)((qx * nq + qy) * nq + qz) * 7 + gi];
                        out[k * n1 + kp] = s;
                    }
            }
        // T2[qx][j k][j' k'] = sum_qy Fy[j][qy] Fy'[j'][qy] T1[qx][qy][k][k']
        int grp = ((d == 0) ? 1 : 0) + ((e == 0) ? 2 : 0);
        double* acc = T2g + (size_t)grp * nq * n2 * n2;
        for (int qx = 0; qx < nq; ++qx)
            for (int j = 0; j < n1; ++j)
                for (int jp = 0; jp < n1; ++jp) {
                    for (int k = 0; k < n1; ++k)
                        for (int kp = 0; kp < n1; ++kp) {
                            double s = 0.0;
                            for (int qy = 0; qy < nq; ++qy)
                                s += Fy[j * nq + qy] * Fyp[jp * nq + qy] *
                                     T1[((size_t)qx * nq + qy) * n2 + k * n1 + kp];
                            acc[((size_t)qx * n2 + j * n1 + k) * n2 + jp * n1 + kp] += s;
                        }
                }
    }
    (void)T2;
    // x direction, once per (row factor, column factor) group
    std::fill(Ke, Ke + (size_t)nl * nl, 0.0);
    for (int grp = 0; grp < 4; ++grp) {
        const double* Fx = (grp & 1) ? t.D.data() : t.L.data();
        const double* Fxp = (grp & 2) ? t.D.data() : t.L.data();
        const double* acc = T2g + (size_t)grp * nq * n2 * n2;
        for (int i = 0; i < n1; ++i)
            for (int ip = 0; ip < n1; ++ip) {
                double c[16];
                for (int qx = 0; qx < nq; ++qx) c[qx] = Fx[i * nq + qx] * Fxp[ip * nq + qx];
                for (int r = 0; r < n2; ++r) {
                    double* row = Ke + (size_t)(i * n2 + r) * nl + ip * n2;
                    for (int cc = 0; cc < n2; ++cc) {
                        double s = 0.0;
                        for (int qx = 0; qx < nq; ++qx) s += c[qx] * acc[((size_t)qx * n2 + r) * n2 + cc];
                        row[cc] += s;
                    }
                }
            }
    }
    for (int a = 0; a < nl; ++a)
        for (int b = a + 1; b < nl; ++b) Ke[(size_t)b * nl + a] = Ke[(size_t)a * nl + b];
    return true;
}

}  // namespace

void reference_tables(int p, int basis, std::vector<double>& L, std::vector<double>& D,
                      std::vector<double>& g, std::vector<double>& w) {
    RefTables t = make_tables(p, basis);
    L = t.L;
    D = t.D;
    g = t.g;
    w = t.wg;
}

void node_elements(const int32_t* l2g, int64_t n_elem, int nl, int64_t n_nodes, std::vector<int64_t>& nstart,
                   std::vector<int32_t>& nel, std::vector<int32_t>& nloc) {
    GIAMG_REQUIRE(n_elem < (int64_t(1) << 31), "too many elements");
    nstart.assign(n_nodes + 1, 0);
    for (int64_t i = 0; i < n_elem * nl; ++i) nstart[l2g[i] + 1]++;
    for (int64_t i = 0; i < n_nodes; ++i) nstart[i + 1] += nstart[i];
    nel.resize(nstart.back());
    nloc.resize(nstart.back());
    std::vector<int64_t> fill(nstart.begin(), nstart.end() - 1);
    for (int64_t e = 0; e < n_elem; ++e)
        for (int a = 0; a < nl; ++a) {
            const int32_t g = l2g[e * nl + a];
            nel[fill[g]] = (int32_t)e;
            nloc[fill[g]] = a;
            fill[g]++;
        }
    for (int64_t i = 0; i < n_nodes; ++i)
        if (nstart[i] == nstart[i + 1])
            throw Error(GIAMG_EINVAL, "node " + std::to_string(i) + " belongs to no element");
}

// ---------------------------------------------------------------------------
// fine-level assembly: symbolic pattern, element matrices, gather by rows
// ---------------------------------------------------------------------------
HostCSR assemble_fine(const std::vector<double>& corners, const int32_t* l2g, int64_t n_elem,
                      int p, int64_t n_nodes, double lambda,
                      const std::vector<uint8_t>& cons, int basis) {
    const int nl = (p + 1) * (p + 1) * (p + 1);
    // node -> (element, local) lists, elements ascending
    std::vector<int64_t> nstart;
    std::vector<int32_t> nel, nloc;
    node_elements(l2g, n_elem, nl, n_nodes, nstart, nel, nloc);

    HostCSR A;
    A.nrows = A.ncols = n_nodes;
    A.rp.assign(n_nodes + 1, 0);
    // symbolic: free rows hold every free node of their elements, constrained
    // rows hold their diagonal only
    std::vector<int64_t> counts(n_nodes, 0);
    parallel_for(n_nodes, 8192, [&](int64_t b, int64_t e) {
        std::vector<int32_t> mark(n_nodes, -1);
        for (int64_t r = b; r < e; ++r) {
            if (cons[r]) { counts[r] = 1; continue; }
            int64_t c = 0;
            for (int64_t s = nstart[r]; s < nstart[r + 1]; ++s) {
                const int32_t* g = l2g + (int64_t)nel[s] * nl;
                for (int a = 0; a < nl; ++a)
                    if (!cons[g[a]] && mark[g[a]] != (int32_t)r) { mark[g[a]] = (int32_t)r; ++c; }
            }
            counts[r] = c;
        }
    });
    for (int64_t r = 0; r < n_nodes; ++r) A.rp[r + 1] = A.rp[r] + counts[r];
    GIAMG_REQUIRE(A.rp.back() < (int64_t(1) << 40), "matrix too large");
    A.ci.resize(A.rp.back());
    A.val.assign(A.rp.back(), 0.0);

    // element matrices (all elements kept: n_elem * nl^2 doubles)
    RefTables t = make_tables(p, basis);
    std::vector<double> Ke((size_t)n_elem * nl * nl);
    std::vector<uint8_t> bad(1, 0);
    parallel_for(n_elem, 16, [&](int64_t b, int64_t e) {
        std::vector<double> work;
        for (int64_t el = b; el < e; ++el)
            if (!element_matrix(t, corners.data() + el * 24, lambda, Ke.data() + (size_t)el * nl * nl, work))
                bad[0] = 1;
    });
    if (bad[0]) throw Error(GIAMG_EINVAL, "non-positive Jacobian determinant in an element");

    // fill columns (sorted) and gather values row by row, elements ascending
    parallel_for(n_nodes, 8192, [&](int64_t b, int64_t e) {
        std::vector<int32_t> pos(n_nodes, -1);
        for (int64_t r = b; r < e; ++r) {
            int64_t o = A.rp[r];
            if (cons[r]) { A.ci[o] = (int32_t)r; A.val[o] = 1.0; continue; }
            int64_t c = 0;
            for (int64_t s = nstart[r]; s < nstart[r + 1]; ++s) {
                const int32_t* g = l2g + (int64_t)nel[s] * nl;
                for (int a = 0; a < nl; ++a)
                    if (!cons[g[a]] && pos[g[a]] != -2) { pos[g[a]] = -2; A.ci[o + c++] = g[a]; }
            }
            std::sort(A.ci.begin() + o, A.ci.begin() + o + c);
            for (int64_t k = 0; k < c; ++k) pos[A.ci[o + k]] = (int32_t)k;
            for (int64_t s = nstart[r]; s < nstart[r + 1]; ++s) {
                const int64_t el = nel[s];
                const int32_t* g = l2g + el * nl;
                const double* row = Ke.data() + ((size_t)el * nl + nloc[s]) * nl;
                for (int a = 0; a < nl; ++a)
                    if (!cons[g[a]]) A.val[o + pos[g[a]]] += row[a];
            }
            for (int64_t k = 0; k < c; ++k) pos[A.ci[o + k]] = -1;
        }
    });
    return A;
}

void quadrature_points(const std::vector<double>& corners, int64_t n_elem, int p, double* xq) {
    RefTables t = make_tables(p, GIAMG_BASIS_NODAL);   // only the Gauss points are used
    const int nq = t.nq, Q = nq * nq * nq;
    for (int64_t e = 0; e < n_elem; ++e) {
        const double* X = corners.data() + e * 24;
        for (int qx = 0; qx < nq; ++qx)
            for (int qy = 0; qy < nq; ++qy)
                for (int qz = 0; qz < nq; ++qz) {
                    double xi[3] = {t.g[qx], t.g[qy], t.g[qz]};
                    double* out = xq + ((size_t)e * Q + (qx * nq + qy) * nq + qz) * 3;
                    out[0] = out[1] = out[2] = 0.0;
                    for (int c = 0; c < 8; ++c) {
                        double N = 1.0;
                        N *= 0.5 * (1 + (((c >> 2) & 1) ? 1 : -1) * xi[0]);
                        N *= 0.5 * (1 + (((c >> 1) & 1) ? 1 : -1) * xi[1]);
                        N *= 0.5 * (1 + ((c & 1) ? 1 : -1) * xi[2]);
                        for (int a = 0; a < 3; ++a) out[a] += N * X[c * 3 + a];
                    }
                }
    }
}

void load_vector(const std::vector<double>& corners, const int32_t* l2g, int64_t n_elem,
                 int p, int64_t n_nodes, const std::vector<uint8_t>& cons,
                 const double* fq, double* b, int basis) {
    RefTables t = make_tables(p, basis);
    const int nq = t.nq, n1 = t.n1, Q = nq * nq * nq, nl = n1 * n1 * n1;
    std::fill(b, b + n_nodes, 0.0);
    std::vector<double> wf(Q);
    for (int64_t e = 0; e < n_elem; ++e) {
        const double* X = corners.data() + e * 24;
        for (int qx = 0; qx < nq; ++qx)
            for (int qy = 0; qy < nq; ++qy)
                for (int qz = 0; qz < nq; ++qz) {
                    double xi[3] = {t.g[qx], t.g[qy], t.g[qz]};
                    double J[3][3];
                    double det = trilinear_jacobian(X, xi, J);
                    int q = (qx * nq + qy) * nq + qz;
                    wf[q] = t.wg[qx] * t.wg[qy] * t.wg[qz] * det * fq[(size_t)e * Q + q];
                }
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n1; ++j)
                for (int k = 0; k < n1; ++k) {
                    double s = 0.0;
                    for (int qx = 0; qx < nq; ++qx)
                        for (int qy = 0; qy < nq; ++qy)
                            for (int qz = 0; qz < nq; ++qz)
                                s += t.L[i * nq + qx] * t.L[j * nq + qy] * t.L[k * nq + qz] *
                                     wf[(qx * nq + qy) * nq + qz];
                    b[l2g[e * nl + lidx(p, i, j, k)]] += s;
                }
    }
    for (int64_t i = 0; i < n_nodes; ++i)
        if (cons[i]) b[i] = 0.0;
}

// ---------------------------------------------------------------------------
// p-coarsening transfer (Algorithms 2-4 and 7): nodal interpolation, or
// injection for the modal basis
// ---------------------------------------------------------------------------
void p_transfer_maps(const std::vector<int32_t>& l2g, int64_t n_elem, int p, int q, int64_t n_fine,
                     const std::vector<uint8_t>& free_mask, std::vector<int32_t>& l2g_next,
                     int64_t& n_coarse, std::vector<double>& I1, int basis) {
    const bool modal = basis == GIAMG_BASIS_MODAL;
    const int nl = (p + 1) * (p + 1) * (p + 1);
    const int ncl = (q + 1) * (q + 1) * (q + 1);
    // Coarse local (a,b,c) is numbered by the fine local node at the nearest
    // lattice positions, pos(a) = floor((2 a p + q) / (2 q)) (a p / q when q
    // divides p; the kept node only numbers the coarse node, P interpolates),
    // or by the same low mode (modal, Algorithm 2).
    std::vector<int> pos(q + 1);
    for (int a = 0; a <= q; ++a) pos[a] = modal ? a : (2 * a * p + q) / (2 * q);
    std::vector<int> extract(ncl);
    for (int a = 0; a <= q; ++a)
        for (int b = 0; b <= q; ++b)
            for (int c = 0; c <= q; ++c) extract[lidx(q, a, b, c)] = lidx(p, pos[a], pos[b], pos[c]);
    auto is_free = [&](int32_t g) { return g >= 0 && free_mask[g]; };
    // collect: kept free fine nodes, sorted, unique; coarse id = rank
    std::vector<int32_t> rank(n_fine, -1);
    for (int64_t e = 0; e < n_elem; ++e)
        for (int a = 0; a < ncl; ++a) {
            int32_t g = l2g[e * nl + extract[a]];
            if (is_free(g)) rank[g] = 0;
        }
    n_coarse = 0;
    for (int64_t g = 0; g < n_fine; ++g)
        if (rank[g] == 0) rank[g] = (int32_t)n_coarse++;
    l2g_next.assign(n_elem * ncl, -1);
    for (int64_t e = 0; e < n_elem; ++e)
        for (int a = 0; a < ncl; ++a) {
            int32_t g = l2g[e * nl + extract[a]];
            l2g_next[e * ncl + a] = is_free(g) ? rank[g] : -1;
        }
    // 1-D factor: interpolation I1[i][a] = l^q_a(xi^p_i) (|.| <= 1e-12 is a
    // structural zero), or the injection I1[a][a] = 1 of the modal basis
    I1.assign((p + 1) * (q + 1), 0.0);
    if (modal) {
        for (int a = 0; a <= q; ++a) I1[a * (q + 1) + a] = 1.0;
    } else {
        std::vector<double> xp, wp, xq, wq;
        gll_points(p, xp, wp);
        gll_points(q, xq, wq);
        for (int i = 0; i <= p; ++i)
            for (int a = 0; a <= q; ++a) {
                double v = lagrange_value(xq, a, xp[i]);
                I1[i * (q + 1) + a] = std::fabs(v) <= 1e-12 ? 0.0 : v;
            }
    }
}

HostCSR p_transfer(const std::vector<int32_t>& l2g, int64_t n_elem, int p, int q,
                   int64_t n_fine, const std::vector<uint8_t>& free_mask,
                   std::vector<int32_t>& l2g_next, int64_t& n_coarse, int basis) {
    const int nl = (p + 1) * (p + 1) * (p + 1);
    const int ncl = (q + 1) * (q + 1) * (q + 1);
    std::vector<double> I1;
    p_transfer_maps(l2g, n_elem, p, q, n_fine, free_mask, l2g_next, n_coarse, I1, basis);
    auto is_free = [&](int32_t g) { return g >= 0 && free_mask[g]; };
    // node -> elements (ascending) for the rows of P
    std::vector<int64_t> nstart(n_fine + 1, 0);
    for (int64_t i = 0; i < n_elem * nl; ++i)
        if (l2g[i] >= 0) nstart[l2g[i] + 1]++;
    for (int64_t i = 0; i < n_fine; ++i) nstart[i + 1] += nstart[i];
    std::vector<int64_t> nel(nstart.back());
    std::vector<int32_t> nloc(nstart.back());
    {
        std::vector<int64_t> fill(nstart.begin(), nstart.end() - 1);
        for (int64_t e = 0; e < n_elem; ++e)
            for (int a = 0; a < nl; ++a) {
                int32_t g = l2g[e * nl + a];
                if (g < 0) continue;
                nel[fill[g]] = e;
                nloc[fill[g]] = a;
                fill[g]++;
            }
    }
    // Row r of P: the union over the node's elements (ascending) of the
    // coarse nodes with a nonzero interpolation weight, the first
    // occurrence of a coarse node kept, then sorted by column.  Two passes
    // over the rows (sizes, then entries into the final arrays), each
    // thread with one scratch row.
    auto build_row = [&](int64_t r, std::vector<std::pair<int32_t, double>>& row) {
        row.clear();
        if (!is_free((int32_t)r)) return;
        for (int64_t t = nstart[r]; t < nstart[r + 1]; ++t) {
            const int64_t el = nel[t];
            const int loc = nloc[t];
            const int i = loc / ((p + 1) * (p + 1)), j = (loc / (p + 1)) % (p + 1), k = loc % (p + 1);
            for (int a = 0; a <= q; ++a) {
                const double va = I1[i * (q + 1) + a];
                if (va == 0.0) continue;
                for (int bb = 0; bb <= q; ++bb) {
                    const double vb = I1[j * (q + 1) + bb];
                    if (vb == 0.0) continue;
                    for (int c = 0; c <= q; ++c) {
                        const double vc = I1[k * (q + 1) + c];
                        if (vc == 0.0) continue;
                        const int32_t gc = l2g_next[el * ncl + lidx(q, a, bb, c)];
                        if (gc < 0) continue;
                        bool dup = false;
                        for (const auto& pr : row)
                            if (pr.first == gc) {
                                dup = true;
                                break;
                            }
                        if (!dup) row.emplace_back(gc, va * vb * vc);
                    }
                }
            }
        }
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                      return x.first < y.first;
                  });
    };
    HostCSR P;
    P.nrows = n_fine;
    P.ncols = n_coarse;
    P.rp.assign(n_fine + 1, 0);
    parallel_for(n_fine, 4096, [&](int64_t b, int64_t e) {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t r = b; r < e; ++r) {
            build_row(r, row);
            P.rp[r + 1] = (int64_t)row.size();
        }
    });
    for (int64_t r = 0; r < n_fine; ++r) P.rp[r + 1] += P.rp[r];
    P.ci.resize(P.rp.back());
    P.val.resize(P.rp.back());
    parallel_for(n_fine, 4096, [&](int64_t b, int64_t e) {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t r = b; r < e; ++r) {
            build_row(r, row);
            int64_t o = P.rp[r];
            for (const auto& pr : row) {
                P.ci[o] = pr.first;
                P.val[o] = pr.second;
                ++o;
            }
        }
    });
    return P;
}

// ---------------------------------------------------------------------------
// smoothed aggregation (Section 2.5): MIS-2 roots by priority, aggregates,
// tentative P, SPAI-0 smoothing
// ---------------------------------------------------------------------------
HostCSR sa_transfer(const HostCSR& A, uint64_t seed, double theta, std::vector<int32_t>& agg,
                    int64_t& n_agg) {
    const int64_t n = A.nrows;
    // strength graph: j is a strong neighbour of i when |a_ij| >= theta
    // sqrt(|a_ii a_jj|); an edge found in either direction is kept in both
    // (the Galerkin rounding may leave a_ij and a_ji a few ulp apart), so
    // the graph is symmetric.  theta = 0 keeps every stored off-diagonal
    // entry, explicit zeros included.
    std::vector<double> adiag(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t s = A.rp[i]; s < A.rp[i + 1]; ++s)
            if (A.ci[s] == i) adiag[i] = std::fabs(A.val[s]);
    auto strong = [&](int64_t i, int64_t s) {
        const int64_t j = A.ci[s];
        return j != i && std::fabs(A.val[s]) >= theta * std::sqrt(adiag[i] * adiag[j]);
    };
    std::vector<int64_t> gp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t s = A.rp[i]; s < A.rp[i + 1]; ++s)
            if (strong(i, s)) { ++gp[i + 1]; ++gp[A.ci[s] + 1]; }
    for (int64_t i = 0; i < n; ++i) gp[i + 1] += gp[i];
    std::vector<int64_t> gfill(gp.begin(), gp.end() - 1);
    std::vector<int32_t> gc(gp[n]);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t s = A.rp[i]; s < A.rp[i + 1]; ++s)
            if (strong(i, s)) {
                gc[gfill[i]++] = A.ci[s];
                gc[gfill[A.ci[s]]++] = (int32_t)i;
            }
    // sort each list and drop the duplicates left by edges found both ways
    std::vector<int64_t> G(n + 1, 0);
    {
        int64_t w = 0;
        for (int64_t i = 0; i < n; ++i) {
            std::sort(gc.begin() + gp[i], gc.begin() + gp[i + 1]);
            const int64_t start = w;
            for (int64_t s = gp[i]; s < gp[i + 1]; ++s)
                if (w == start || gc[w - 1] != gc[s]) gc[w++] = gc[s];
            G[i + 1] = w;
        }
        gc.resize(w);
    }
    std::vector<uint64_t> h(n);
    for (int64_t i = 0; i < n; ++i) h[i] = splitmix64(seed, (uint64_t)i);
    auto higher = [&](int64_t a, int64_t b) {   // priority(a) > priority(b)
        return h[a] != h[b] ? h[a] > h[b] : a > b;
    };
    std::vector<int64_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), higher);
    // greedy MIS of the distance-2 strength graph
    std::vector<uint8_t> blocked(n, 0), is_root(n, 0);
    for (int64_t v : order) {
        if (blocked[v]) continue;
        is_root[v] = 1;
        blocked[v] = 1;
        for (int64_t s = G[v]; s < G[v + 1]; ++s) {
            int64_t u = gc[s];
            blocked[u] = 1;
            for (int64_t t = G[u]; t < G[u + 1]; ++t) blocked[gc[t]] = 1;
        }
    }
    agg.assign(n, -1);
    std::vector<int64_t> root_of(n, -1);
    n_agg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (is_root[v]) { agg[v] = (int32_t)n_agg++; root_of[v] = v; }
    for (int64_t v = 0; v < n; ++v) {
        if (!is_root[v]) continue;
        for (int64_t s = G[v]; s < G[v + 1]; ++s) {
            int64_t u = gc[s];
            agg[u] = agg[v];
            root_of[u] = v;
        }
    }
    std::vector<int32_t> first(agg);
    std::vector<int64_t> first_root(root_of);
    for (int64_t v = 0; v < n; ++v) {
        if (first[v] >= 0) continue;
        int64_t best = -1;
        for (int64_t s = G[v]; s < G[v + 1]; ++s) {
            int64_t u = gc[s];
            if (first[u] < 0) continue;
            int64_t r = first_root[u];
            if (best < 0 || higher(r, best)) best = r;
        }
        if (best < 0) throw Error(GIAMG_EINVAL, "aggregation left a node unassigned");
        agg[v] = first[best];
    }
    // SPAI-0 weights and P = (I - diag(m) A) T on pattern(T) u pattern(A T)
    HostCSR P;
    P.nrows = n;
    P.ncols = n_agg;
    P.rp.assign(n + 1, 0);
    std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
    parallel_for(n, 1024, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            double aii = 0.0, sq = 0.0;
            for (int64_t s = A.rp[i]; s < A.rp[i + 1]; ++s) {
                if (A.ci[s] == i) aii = A.val[s];
                sq += A.val[s] * A.val[s];
            }
            double m = aii / sq;
            auto& row = rows[i];
            auto add = [&row](int32_t c, double v) {
                for (auto& pr : row)
                    if (pr.first == c) { pr.second += v; return; }
                row.emplace_back(c, v);
            };
            // (A T)_ij summed over the row in column order, then T - m (A T)
            std::vector<std::pair<int32_t, double>> at;
            for (int64_t s = A.rp[i]; s < A.rp[i + 1]; ++s) {
                int32_t c = agg[A.ci[s]];
                bool found = false;
                for (auto& pr : at)
                    if (pr.first == c) { pr.second += A.val[s]; found = true; break; }
                if (!found) at.emplace_back(c, A.val[s]);
            }
            add(agg[i], 0.0);
            for (auto& pr : at) add(pr.first, 0.0);
            for (auto& pr : row) {
                double tv = (pr.first == agg[i]) ? 1.0 : 0.0;
                double atv = 0.0;
                for (auto& q : at)
                    if (q.first == pr.first) { atv = q.second; break; }
                pr.second = tv - m * atv;
            }
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                          return x.first < y.first;
                      });
        }
    });
    for (int64_t r = 0; r < n; ++r) P.rp[r + 1] = P.rp[r] + (int64_t)rows[r].size();
    P.ci.resize(P.rp.back());
    P.val.resize(P.rp.back());
    for (int64_t r = 0; r < n; ++r) {
        int64_t o = P.rp[r];
        for (auto& pr : rows[r]) { P.ci[o] = pr.first; P.val[o] = pr.second; ++o; }
    }
    return P;
}

HostCSR transpose(const HostCSR& M) {
    HostCSR T;
    T.nrows = M.ncols;
    T.ncols = M.nrows;
    T.rp.assign(T.nrows + 1, 0);
    for (int64_t k = 0; k < M.nnz(); ++k) T.rp[M.ci[k] + 1]++;
    for (int64_t i = 0; i < T.nrows; ++i) T.rp[i + 1] += T.rp[i];
    T.ci.resize(M.nnz());
    T.val.resize(M.nnz());
    std::vector<int64_t> fill(T.rp.begin(), T.rp.end() - 1);
    for (int64_t r = 0; r < M.nrows; ++r)           // rows ascending -> columns ascending
        for (int64_t k = M.rp[r]; k < M.rp[r + 1]; ++k) {
            int64_t o = fill[M.ci[k]]++;
            T.ci[o] = (int32_t)r;
            T.val[o] = M.val[k];
        }
    return T;
}

// Cholesky A = L L^T, then A^-1 = L^-T L^-1 column by column.  Every sum
// runs over k in ascending order, so the result does not depend on the
// thread count.  The factor is computed column by column by one team of
// threads (rows dealt out cyclically, a barrier per column) instead of a
// thread launch per column; the solves skip the leading zeros of e_c (the
// terms they drop are exact zeros) and read L^T row-wise.
bool spd_inverse(const std::vector<double>& A, int64_t n, std::vector<double>& inv) {
    std::vector<double> L(A);
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)hw, 16, n / 32}));
    std::atomic<int64_t> arrived{0};
    std::atomic<bool> ok{true};
    auto factor = [&](int t) {
        for (int64_t j = 0; j < n; ++j) {
            double d = L[j * n + j];
            for (int64_t k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
            if (!(d > 0.0)) {
                ok = false;
            } else {
                d = std::sqrt(d);
                for (int64_t i = j + 1 + t; i < n; i += nt) {
                    double s = L[i * n + j];
                    for (int64_t k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
                    L[i * n + j] = s / d;
                }
            }
            arrived.fetch_add(1);   // column j done: the next reads it
            while (arrived.load() < (j + 1) * nt) std::this_thread::yield();
            if (!ok) return;
            // every thread has read the diagonal entry of column j; later
            // columns do not read it, the solves do
            if (t == 0) L[j * n + j] = d;
        }
    };
    {
        std::vector<std::thread> team;
        for (int t = 1; t < nt; ++t) team.emplace_back(factor, t);
        factor(0);
        for (auto& th : team) th.join();
    }
    if (!ok) return false;
    std::vector<double> U((size_t)(n * n));   // U = L^T, row-major
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < n; ++k) U[k * n + i] = L[i * n + k];
    inv.assign(n * n, 0.0);
    parallel_for(n, 8, [&](int64_t b, int64_t e) {
        std::vector<double> y(n), z(n);
        for (int64_t c = b; c < e; ++c) {
            std::fill(y.begin(), y.begin() + c, 0.0);
            for (int64_t i = c; i < n; ++i) {          // L y = e_c (y_i = 0 for i < c)
                double s = (i == c) ? 1.0 : 0.0;
                for (int64_t k = c; k < i; ++k) s -= L[i * n + k] * y[k];
                y[i] = s / L[i * n + i];
            }
            for (int64_t i = n - 1; i >= 0; --i) {     // L^T z = y
                double s = y[i];
                for (int64_t k = i + 1; k < n; ++k) s -= U[i * n + k] * z[k];
                z[i] = s / U[i * n + i];
            }
            for (int64_t i = 0; i < n; ++i) inv[i * n + c] = z[i];
        }
    });
    // symmetrise exactly
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double v = 0.5 * (inv[i * n + j] + inv[j * n + i]);
            inv[i * n + j] = inv[j * n + i] = v;
        }
    return true;
}

}  // namespace giamg
