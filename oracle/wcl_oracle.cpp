// Plain FP64 CPU oracle for the Wilson-clover RAS / nested-BiCGStab solver.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
// its Python binding) includes, links, imports or runs this file; only the
// test suite, the smoke check and the CPU-baseline leg of the benchmark do.
// It shares no code, header, table or constant with the HIP path.
//
// Everything is std::complex<double>, plain loops over sites, explicit 4x4
// gamma matrices and explicit 3x3 colour matrices, written for readability
// against the paper, not for speed (OpenMP over sites only).
//
// What each part follows:
//   * the linear system D phi = eta ........................ Sec. 1, Eq. (1)
//   * the O(a)-improved Wilson (clover) operator ........... Sec. 1 / Sec. 5
//     (the paper names the operator, kappa and c_SW but prints no formula;
//      the standard kappa-normalised form below is the reading used, see
//      D_at below)
//   * Dirichlet-restricted domain operator D_{Omega'} ...... Sec. 2
//   * the RAS iteration (projection, domain solve,
//     restriction, sum, phi += v, r -= D v) ................ Sec. 2, Algorithm 1
//   * fixed-iteration domain solver (read as minimal
//     residual, N_dominv steps, zero start) ................ Sec. 2
//     other readings: block Jacobi with the site term as
//     the diagonal, and BiCGStab truncated to N_dominv
//     iterations ........................................... Sec. 2
//   * additive Schwarz (whole extended solutions summed,
//     Richardson refinement) and multiplicative Schwarz
//     (two colours of domains, residual updated between) ... Sec. 1-2
//   * even-odd reduction to the Schur complement on the
//     even sites (not in the paper; an accelerator of the
//     same solve, using the 12x12 site-term inverse)
//   * BiCGStab, right preconditioning D K chi = eta ......... Sec. 2, Eq. (3)
//   * mixed-precision nested BiCGStab (outer solver whose
//     preconditioner is an inner BiCGStab) ................. Sec. 3
//     (the oracle runs both levels in FP64)
//
// parity pinned by: free-field plane-wave closed form, gamma5-hermiticity,
// gauge covariance, uniform abelian field closed form for the clover term,
// dense brute force on 2^4, the Eq. (2) identity for RAS, the exact-block RAS
// invariant, BiCGStab against dense LU, the extended-domain membership rule
// of Sec. 4, the Neumann series of block Jacobi, BiCGStab's Galerkin and
// minimal-residual conditions, the dense additive-Schwarz identity, the dense
// error propagator of the multiplicative iteration and the dense Schur
// complement (see tests/test_oracle_*.py).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

using cplx = std::complex<double>;

namespace {

const cplx I1(0.0, 1.0);

// ---------------------------------------------------------------- gammas --
// Chiral basis (the paper does not fix one):
//   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = x, y, z)
//   gamma_t = [[0, -1], [-1, 0]]
struct Dirac {
    cplx g[4][4][4];          // g[mu][row][col]
    cplx sigma[4][4][4][4];   // sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu]
};

Dirac make_dirac() {
    Dirac d{};
    cplx pauli[3][2][2] = {
        {{0.0, 1.0}, {1.0, 0.0}},
        {{0.0, -I1}, {I1, 0.0}},
        {{1.0, 0.0}, {0.0, -1.0}},
    };
    for (int mu = 0; mu < 4; ++mu)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) d.g[mu][a][b] = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                d.g[k][a][2 + b] = -I1 * pauli[k][a][b];
                d.g[k][2 + a][b] = I1 * pauli[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        d.g[3][a][2 + a] = -1.0;
        d.g[3][2 + a][a] = -1.0;
    }
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx c = 0.0;
                    for (int k = 0; k < 4; ++k)
                        c += d.g[mu][a][k] * d.g[nu][k][b] - d.g[nu][a][k] * d.g[mu][k][b];
                    d.sigma[mu][nu][a][b] = 0.5 * I1 * c;
                }
    return d;
}

const Dirac DIRAC = make_dirac();

// ------------------------------------------------------------ su(3) ------
struct M3 {
    cplx m[3][3];
};

M3 mul(const M3& A, const M3& B) {
    M3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < 3; ++k) s += A.m[i][k] * B.m[k][j];
            C.m[i][j] = s;
        }
    return C;
}

M3 dag(const M3& A) {
    M3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.m[i][j] = std::conj(A.m[j][i]);
    return C;
}

M3 add(const M3& A, const M3& B) {
    M3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][j] + B.m[i][j];
    return C;
}

// ---------------------------------------------------------- lattice ------
struct Lattice {
    int L[4];
    int bc[4];       // +1 periodic, -1 antiperiodic (fermion hops only)
    int64_t V;
    const cplx* U;   // [V][4][3][3], caller-owned
    std::vector<cplx> clover;  // [V][12][12] when precomputed

    int64_t index(const int c[4]) const {
        return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
    }
    void coords(int64_t i, int c[4]) const {
        for (int mu = 0; mu < 4; ++mu) {
            c[mu] = (int)(i % L[mu]);
            i /= L[mu];
        }
    }
    // neighbour of site i shifted by +-1 in direction mu; *phase gets the
    // fermion boundary phase picked up when the hop wraps round the lattice.
    int64_t hop(int64_t i, int mu, int dir, double* phase) const {
        int c[4];
        coords(i, c);
        int n = c[mu] + dir;
        double ph = 1.0;
        if (n < 0) { n += L[mu]; ph = bc[mu]; }
        if (n >= L[mu]) { n -= L[mu]; ph = bc[mu]; }
        c[mu] = n;
        if (phase) *phase = ph;
        return index(c);
    }
    int64_t shift(int64_t i, int mu, int dir) const { return hop(i, mu, dir, nullptr); }
    M3 link(int64_t i, int mu) const {
        M3 A;
        const cplx* p = U + ((i * 4 + mu) * 9);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A.m[a][b] = p[a * 3 + b];
        return A;
    }
};

// Sum of the four plaquette leaves in the (mu, nu) plane at site x.
M3 leaves(const Lattice& lat, int64_t x, int mu, int nu) {
    int64_t xpm = lat.shift(x, mu, +1), xpn = lat.shift(x, nu, +1);
    int64_t xmm = lat.shift(x, mu, -1), xmn = lat.shift(x, nu, -1);
    int64_t xpn_mm = lat.shift(xpn, mu, -1);
    int64_t xmm_mn = lat.shift(xmm, nu, -1);
    int64_t xpm_mn = lat.shift(xpm, nu, -1);
    M3 q1 = mul(mul(lat.link(x, mu), lat.link(xpm, nu)),
                mul(dag(lat.link(xpn, mu)), dag(lat.link(x, nu))));
    M3 q2 = mul(mul(lat.link(x, nu), dag(lat.link(xpn_mm, mu))),
                mul(dag(lat.link(xmm, nu)), lat.link(xmm, mu)));
    M3 q3 = mul(mul(dag(lat.link(xmm, mu)), dag(lat.link(xmm_mn, nu))),
                mul(lat.link(xmm_mn, mu), lat.link(xmn, nu)));
    M3 q4 = mul(mul(dag(lat.link(xmn, nu)), lat.link(xmn, mu)),
                mul(lat.link(xpm_mn, nu), dag(lat.link(x, mu))));
    return add(add(q1, q2), add(q3, q4));
}

// Fhat_{mu nu} = (1/8) [ (Q - Q^dag) - (1/3) Tr(Q - Q^dag) ]
M3 field_strength(const Lattice& lat, int64_t x, int mu, int nu) {
    M3 Q = leaves(lat, x, mu, nu);
    M3 A;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A.m[a][b] = Q.m[a][b] - std::conj(Q.m[b][a]);
    cplx tr = A.m[0][0] + A.m[1][1] + A.m[2][2];
    for (int a = 0; a < 3; ++a) A.m[a][a] -= tr / 3.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A.m[a][b] *= 0.125;
    return A;
}

// C(x) = i sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x), a 12x12 matrix with
// row/column index 3*spin + colour.
void clover_site(const Lattice& lat, int64_t x, cplx* C /*[12][12]*/) {
    for (int k = 0; k < 144; ++k) C[k] = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            M3 F = field_strength(lat, x, mu, nu);
            for (int s = 0; s < 4; ++s)
                for (int sp = 0; sp < 4; ++sp) {
                    cplx sg = I1 * DIRAC.sigma[mu][nu][s][sp];
                    if (sg == 0.0) continue;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            C[(3 * s + a) * 12 + 3 * sp + b] += sg * F.m[a][b];
                }
        }
}

const cplx* clover_of(const Lattice& lat, int64_t x, cplx* tmp) {
    if (!lat.clover.empty()) return lat.clover.data() + x * 144;
    clover_site(lat, x, tmp);
    return tmp;
}

// Adds coef * Gam * (M psi_site) to out, Gam a 4x4 spin matrix and M a colour
// matrix acting on each spin component.
void add_spin_colour(const cplx (&Gam)[4][4], const M3& M, const cplx* psi, cplx coef, cplx* out) {
    cplx mpsi[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx t = 0.0;
            for (int b = 0; b < 3; ++b) t += M.m[a][b] * psi[3 * s + b];
            mpsi[s][a] = t;
        }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx t = 0.0;
            for (int sp = 0; sp < 4; ++sp) t += Gam[s][sp] * mpsi[sp][a];
            out[3 * s + a] += coef * t;
        }
}

// Spinor accessor: the 12 components of the field at a global site, or
// nullptr when that site is outside the operator's domain.
using Fetch = std::function<const cplx*(int64_t)>;

// (D psi)(x) for the kappa-normalised O(a)-improved Wilson operator:
//   (D psi)(x) = psi(x) + c_sw kappa C(x) psi(x)
//      - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
//                     + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
// A hop whose target the accessor reports as outside (nullptr) is dropped:
// that is the Dirichlet restriction of Sec. 2.
void D_at(const Lattice& lat, double kappa, double csw, const Fetch& fetch, int64_t x, cplx* out /*[12]*/) {
    cplx tmp[144];
    const cplx* C = clover_of(lat, x, tmp);
    const cplx* px = fetch(x);
    for (int i = 0; i < 12; ++i) {
        cplx c = 0.0;
        for (int j = 0; j < 12; ++j) c += C[i * 12 + j] * px[j];
        out[i] = px[i] + csw * kappa * c;
    }
    cplx one_minus[4][4], one_plus[4][4];
    for (int mu = 0; mu < 4; ++mu) {
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx id = (a == b) ? 1.0 : 0.0;
                one_minus[a][b] = id - DIRAC.g[mu][a][b];
                one_plus[a][b] = id + DIRAC.g[mu][a][b];
            }
        double ph;
        int64_t xf = lat.hop(x, mu, +1, &ph);
        if (const cplx* pf = fetch(xf)) add_spin_colour(one_minus, lat.link(x, mu), pf, -kappa * ph, out);
        int64_t xb = lat.hop(x, mu, -1, &ph);
        if (const cplx* pb = fetch(xb)) add_spin_colour(one_plus, dag(lat.link(xb, mu)), pb, -kappa * ph, out);
    }
}

void apply_D(const Lattice& lat, double kappa, double csw, const cplx* psi, cplx* out) {
    Fetch whole = [psi](int64_t y) { return psi + y * 12; };
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < lat.V; ++x) D_at(lat, kappa, csw, whole, x, out + x * 12);
}

// The hopping part of D alone at x (every term of D_at but the site term):
//   out = -kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ],
// hops to sites the accessor reports as outside dropped.
void hops_at(const Lattice& lat, double kappa, const Fetch& fetch, int64_t x, cplx* out /*[12]*/) {
    for (int i = 0; i < 12; ++i) out[i] = 0.0;
    cplx one_minus[4][4], one_plus[4][4];
    for (int mu = 0; mu < 4; ++mu) {
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx id = (a == b) ? 1.0 : 0.0;
                one_minus[a][b] = id - DIRAC.g[mu][a][b];
                one_plus[a][b] = id + DIRAC.g[mu][a][b];
            }
        double ph;
        int64_t xf = lat.hop(x, mu, +1, &ph);
        if (const cplx* pf = fetch(xf)) add_spin_colour(one_minus, lat.link(x, mu), pf, -kappa * ph, out);
        int64_t xb = lat.hop(x, mu, -1, &ph);
        if (const cplx* pb = fetch(xb)) add_spin_colour(one_plus, dag(lat.link(xb, mu)), pb, -kappa * ph, out);
    }
}

// The site term A(x) = 1 + c_sw kappa C(x) as a 12x12 matrix.
void site_term(const Lattice& lat, double kappa, double csw, int64_t x, cplx* A /*[144]*/) {
    cplx tmp[144];
    const cplx* C = clover_of(lat, x, tmp);
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) A[i * 12 + j] = (i == j ? 1.0 : 0.0) + csw * kappa * C[i * 12 + j];
}

// Inverse of a general n x n complex matrix by Gauss-Jordan elimination with
// partial pivoting; false if a pivot vanishes.
bool invert(int n, const cplx* A, cplx* Ainv) {
    std::vector<cplx> M(A, A + n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(M[r * n + c]) > std::abs(M[piv * n + c])) piv = r;
        if (std::abs(M[piv * n + c]) == 0.0) return false;
        if (piv != c)
            for (int j = 0; j < n; ++j) {
                std::swap(M[c * n + j], M[piv * n + j]);
                std::swap(Ainv[c * n + j], Ainv[piv * n + j]);
            }
        const cplx inv = 1.0 / M[c * n + c];
        for (int j = 0; j < n; ++j) {
            M[c * n + j] *= inv;
            Ainv[c * n + j] *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const cplx f = M[r * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                M[r * n + j] -= f * M[c * n + j];
                Ainv[r * n + j] -= f * Ainv[c * n + j];
            }
        }
    }
    return true;
}

// y = M x for a 12x12 matrix and a 12-component site vector.
void matvec12(const cplx* M, const cplx* x, cplx* y) {
    for (int i = 0; i < 12; ++i) {
        cplx t = 0.0;
        for (int j = 0; j < 12; ++j) t += M[i * 12 + j] * x[j];
        y[i] = t;
    }
}

// ------------------------------------------------------ BLAS-1 (FP64) ----
cplx dot(const std::vector<cplx>& a, const std::vector<cplx>& b) {
    cplx s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += std::conj(a[i]) * b[i];
    return s;
}
double norm2(const std::vector<cplx>& a) {
    double s = 0.0;
    for (const cplx& z : a) s += std::norm(z);
    return s;
}

// ------------------------------------------------------ domains ----------
// Blocks Omega_i tile the lattice by b starting at the origin; Omega'_i grows
// each block by s sites per side in every direction the block does not span.
struct Decomp {
    int b[4], s[4], e[4], nb[4];
    int64_t nblocks;
    int64_t ext_volume;
};

bool make_decomp(const Lattice& lat, const int b[4], int s, Decomp* d) {
    d->nblocks = 1;
    d->ext_volume = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (b[mu] <= 0 || lat.L[mu] % b[mu] != 0) return false;
        d->b[mu] = b[mu];
        d->s[mu] = (b[mu] < lat.L[mu]) ? s : 0;
        d->e[mu] = b[mu] + 2 * d->s[mu];
        if (d->e[mu] > lat.L[mu]) return false;
        d->nb[mu] = lat.L[mu] / b[mu];
        d->nblocks *= d->nb[mu];
        d->ext_volume *= d->e[mu];
    }
    return true;
}

void block_origin(const Decomp& d, int64_t blk, int o[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        o[mu] = (int)(blk % d.nb[mu]) * d.b[mu];
        blk /= d.nb[mu];
    }
}

// The global sites of Omega'_i, listed in lexicographic order of their local
// coordinates l_mu = x_mu - o_mu + s_mu (mod L_mu).
std::vector<int64_t> ext_sites(const Lattice& lat, const Decomp& d, int64_t blk) {
    int o[4];
    block_origin(d, blk, o);
    std::vector<int64_t> out;
    out.reserve(d.ext_volume);
    for (int l3 = 0; l3 < d.e[3]; ++l3)
        for (int l2 = 0; l2 < d.e[2]; ++l2)
            for (int l1 = 0; l1 < d.e[1]; ++l1)
                for (int l0 = 0; l0 < d.e[0]; ++l0) {
                    int l[4] = {l0, l1, l2, l3}, c[4];
                    for (int mu = 0; mu < 4; ++mu)
                        c[mu] = ((o[mu] - d.s[mu] + l[mu]) % lat.L[mu] + lat.L[mu]) % lat.L[mu];
                    out.push_back(lat.index(c));
                }
    return out;
}

bool owned(const Lattice& lat, const Decomp& d, int64_t blk, int64_t x) {
    int o[4], c[4];
    block_origin(d, blk, o);
    lat.coords(x, c);
    for (int mu = 0; mu < 4; ++mu)
        if (c[mu] < o[mu] || c[mu] >= o[mu] + d.b[mu]) return false;
    return true;
}

// Position of global site y inside Omega'_blk (local lexicographic order of
// l_mu = x_mu - o_mu + s_mu mod L_mu), or -1 if y is not in the set.
int64_t ext_local(const Lattice& lat, const Decomp& d, const int o[4], int64_t y) {
    int c[4];
    lat.coords(y, c);
    int64_t k = 0, stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        int l = ((c[mu] - o[mu] + d.s[mu]) % lat.L[mu] + lat.L[mu]) % lat.L[mu];
        if (l >= d.e[mu]) return -1;
        k += stride * l;
        stride *= d.e[mu];
    }
    return k;
}

// Operator D_{Omega'} = P D P^T on the extended block blk: a principal
// submatrix of D, i.e. every hop whose target is outside Omega' is dropped.
struct BlockOp {
    const Lattice& lat;
    const Decomp& d;
    int o[4];
    std::vector<int64_t> sites;
    BlockOp(const Lattice& l, const Decomp& dd, int64_t blk) : lat(l), d(dd), sites(ext_sites(l, dd, blk)) {
        block_origin(dd, blk, o);
    }
    void apply(double kappa, double csw, const std::vector<cplx>& in, std::vector<cplx>& out) {
        out.resize(in.size());
        Fetch inside = [&](int64_t y) -> const cplx* {
            int64_t k = ext_local(lat, d, o, y);
            return k < 0 ? nullptr : in.data() + k * 12;
        };
        for (size_t k = 0; k < sites.size(); ++k) D_at(lat, kappa, csw, inside, sites[k], &out[k * 12]);
    }
};

// ------------------------------------------------------ BiCGStab ---------
// van der Vorst BiCGStab with right preconditioning (Eq. (3)):
// solves A y = b with y = K chi, K == nullptr meaning K = 1.
// Stops on the recursive residual |r| <= tol |b|.
using VecOp = std::function<void(const std::vector<cplx>&, std::vector<cplx>&)>;

struct SolveInfo {
    int iters;
    int restarts;
    double rel_resid;   // recursive residual / |b|
    int converged;
};

SolveInfo bicgstab(const VecOp& A, const VecOp* K, const std::vector<cplx>& b, std::vector<cplx>& x,
                   double tol, int max_iter) {
    const size_t n = b.size();
    SolveInfo info{0, 0, 0.0, 0};
    double bnorm = std::sqrt(norm2(b));
    x.assign(n, 0.0);
    if (bnorm == 0.0) {
        info.converged = 1;
        return info;
    }
    std::vector<cplx> r = b, rhat = b, p(n, 0.0), v(n, 0.0), s(n), t(n), phat(n), shat(n);
    cplx rho_old = 1.0, alpha = 1.0, omega = 1.0;
    double rnorm = bnorm;
    for (int it = 0; it < max_iter; ++it) {
        cplx rho = dot(rhat, r);
        if (std::abs(rho) < 1e-30 * std::sqrt(norm2(rhat)) * rnorm) {
            // breakdown: restart the shadow residual from the current r
            rhat = r;
            p.assign(n, 0.0);
            v.assign(n, 0.0);
            rho_old = alpha = omega = 1.0;
            rho = dot(rhat, r);
            ++info.restarts;
        }
        cplx beta = (rho / rho_old) * (alpha / omega);
        for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        if (K) (*K)(p, phat); else phat = p;
        A(phat, v);
        cplx rv = dot(rhat, v);
        alpha = rho / rv;
        for (size_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double snorm = std::sqrt(norm2(s));
        if (snorm <= tol * bnorm) {
            for (size_t i = 0; i < n; ++i) x[i] += alpha * phat[i];
            r = s;
            rnorm = snorm;
            info.iters = it + 1;
            info.rel_resid = rnorm / bnorm;
            info.converged = 1;
            return info;
        }
        if (K) (*K)(s, shat); else shat = s;
        A(shat, t);
        double tt = norm2(t);
        omega = (tt > 0.0) ? dot(t, s) / tt : cplx(0.0);
        for (size_t i = 0; i < n; ++i) x[i] += alpha * phat[i] + omega * shat[i];
        for (size_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rho_old = rho;
        rnorm = std::sqrt(norm2(r));
        info.iters = it + 1;
        info.rel_resid = rnorm / bnorm;
        if (rnorm <= tol * bnorm) {
            info.converged = 1;
            return info;
        }
        if (omega == 0.0) {
            rhat = r;
            p.assign(n, 0.0);
            v.assign(n, 0.0);
            rho_old = alpha = omega = 1.0;
            ++info.restarts;
        }
    }
    return info;
}

// ------------------------------------------------------ domain solvers ---
// Minimal residual, zero start, exactly n steps (no early exit):
//   q = D rho; alpha = <q,rho>/<q,q>; x += alpha rho; rho -= alpha q.
void mr_solve(BlockOp& op, double kappa, double csw, const std::vector<cplx>& b, std::vector<cplx>& x, int n) {
    const size_t m = b.size();
    std::vector<cplx> rho = b, q(m);
    x.assign(m, 0.0);
    for (int k = 0; k < n; ++k) {
        op.apply(kappa, csw, rho, q);
        double qq = norm2(q);
        if (qq == 0.0) break;
        cplx alpha = dot(q, rho) / qq;
        for (size_t i = 0; i < m; ++i) {
            x[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
}

// Block Jacobi, zero start, exactly n steps: x <- x + A^{-1} (b - D x), A the
// site term of each site of the domain (the diagonal blocks of D_{Omega'}).
void jacobi_solve(BlockOp& op, double kappa, double csw, const std::vector<cplx>& b, std::vector<cplx>& x, int n) {
    const size_t m = b.size();
    std::vector<cplx> Ainv(op.sites.size() * 144), Dx(m), r(m);
    for (size_t k = 0; k < op.sites.size(); ++k) {
        cplx A[144];
        site_term(op.lat, kappa, csw, op.sites[k], A);
        invert(12, A, &Ainv[k * 144]);
    }
    x.assign(m, 0.0);
    for (int it = 0; it < n; ++it) {
        op.apply(kappa, csw, x, Dx);
        for (size_t i = 0; i < m; ++i) r[i] = b[i] - Dx[i];
        for (size_t k = 0; k < op.sites.size(); ++k) {
            cplx z[12];
            matvec12(&Ainv[k * 144], &r[k * 12], z);
            for (int i = 0; i < 12; ++i) x[k * 12 + i] += z[i];
        }
    }
}

// BiCGStab truncated to exactly n iterations from zero, no restarts and no
// early exit.  A vanishing denominator makes its coefficient zero:
// alpha = 0 when <rhat, v> = 0, omega = 0 when |t| = 0, beta = 0 when
// rho_old = 0 or omega = 0 (so a zero right-hand side gives x = 0).
void bicgstab_fixed(BlockOp& op, double kappa, double csw, const std::vector<cplx>& b, std::vector<cplx>& x, int n) {
    const size_t m = b.size();
    std::vector<cplx> r = b, rhat = b, p(m, 0.0), v(m, 0.0), s(m), t(m);
    x.assign(m, 0.0);
    cplx rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (int it = 0; it < n; ++it) {
        const cplx rho = dot(rhat, r);
        const cplx beta = (rho_old != 0.0 && omega != 0.0) ? (rho / rho_old) * (alpha / omega) : cplx(0.0);
        for (size_t i = 0; i < m; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        op.apply(kappa, csw, p, v);
        const cplx rv = dot(rhat, v);
        alpha = (rv != 0.0) ? rho / rv : cplx(0.0);
        for (size_t i = 0; i < m; ++i) s[i] = r[i] - alpha * v[i];
        op.apply(kappa, csw, s, t);
        const double tt = norm2(t);
        omega = (tt > 0.0) ? dot(t, s) / tt : cplx(0.0);
        for (size_t i = 0; i < m; ++i) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rho_old = rho;
    }
}

enum { DOM_MR = 0, DOM_JACOBI = 1, DOM_BICGSTAB = 2 };
enum { SCH_RAS = 0, SCH_AS = 1, SCH_SAP = 2 };

struct RasParams {
    int b[4];
    int s;
    int n_ras;
    int n_dominv;
    int exact;     // 1: domain solve by BiCGStab to 1e-14 instead of the fixed-iteration solver
    int solver;    // DOM_*: the fixed-iteration domain solver (Sec. 2)
    int schwarz;   // SCH_*: restricted additive (Algorithm 1), additive, multiplicative
};

// Colour of domain blk for the multiplicative iteration: parity of the sum of
// its block coordinates.
int block_colour(const Decomp& d, int64_t blk) {
    int c = 0;
    for (int mu = 0; mu < 4; ++mu) {
        c += (int)(blk % d.nb[mu]);
        blk /= d.nb[mu];
    }
    return c & 1;
}

// Solves every domain of the given colour (-1: all) on the residual r and
// sums the results into v: the restriction R_{Omega_i} (owned sites only) for
// the restricted iterations, the whole extended solution (overlaps add up)
// for the additive one.
void domain_pass(const Lattice& lat, const Decomp& d, const RasParams& P, double kappa, double csw,
                 const std::vector<cplx>& r, int colour, std::vector<cplx>& v) {
    std::fill(v.begin(), v.end(), cplx(0.0));
    std::vector<std::vector<cplx>> sol(d.nblocks);
#pragma omp parallel for schedule(dynamic)
    for (int64_t blk = 0; blk < d.nblocks; ++blk) {
        if (colour >= 0 && block_colour(d, blk) != colour) continue;
        BlockOp op(lat, d, blk);
        const std::vector<int64_t>& sites = op.sites;
        // projection r_{Omega'} = P r
        std::vector<cplx> rb(sites.size() * 12);
        for (size_t k = 0; k < sites.size(); ++k)
            for (int i = 0; i < 12; ++i) rb[k * 12 + i] = r[sites[k] * 12 + i];
        // domain solve with the Dirichlet boundary condition
        if (P.exact) {
            VecOp A = [&](const std::vector<cplx>& a, std::vector<cplx>& o) {
                o.resize(a.size());
                op.apply(kappa, csw, a, o);
            };
            bicgstab(A, nullptr, rb, sol[blk], 1e-14, 100000);
        } else if (P.solver == DOM_JACOBI) {
            jacobi_solve(op, kappa, csw, rb, sol[blk], P.n_dominv);
        } else if (P.solver == DOM_BICGSTAB) {
            bicgstab_fixed(op, kappa, csw, rb, sol[blk], P.n_dominv);
        } else {
            mr_solve(op, kappa, csw, rb, sol[blk], P.n_dominv);
        }
    }
    // the sum over domains, in domain order
    for (int64_t blk = 0; blk < d.nblocks; ++blk) {
        if (sol[blk].empty()) continue;
        std::vector<int64_t> sites = ext_sites(lat, d, blk);
        for (size_t k = 0; k < sites.size(); ++k)
            if (P.schwarz == SCH_AS || owned(lat, d, blk, sites[k]))
                for (int i = 0; i < 12; ++i) v[sites[k] * 12 + i] += sol[blk][k * 12 + i];
    }
}

// Algorithm 1: phi = K_RAS eta, and the other Schwarz iterations of Sec. 1-2:
// the additive one (the whole extended solutions summed, refined by the same
// Richardson update) and the multiplicative one (each sweep solves the
// colour-0 domains, updates phi and r, then the colour-1 domains).
bool ras(const Lattice& lat, const RasParams& P, double kappa, double csw,
         const std::vector<cplx>& eta, std::vector<cplx>& phi) {
    Decomp d;
    if (!make_decomp(lat, P.b, P.s, &d)) return false;
    const int64_t n = lat.V * 12;
    std::vector<cplx> r = eta, v(n), Dv(n);
    phi.assign(n, 0.0);
    const int passes = P.schwarz == SCH_SAP ? 2 : 1;
    for (int j = 0; j < P.n_ras; ++j)
        for (int c = 0; c < passes; ++c) {
            domain_pass(lat, d, P, kappa, csw, r, P.schwarz == SCH_SAP ? c : -1, v);
            for (int64_t i = 0; i < n; ++i) phi[i] += v[i];
            apply_D(lat, kappa, csw, v.data(), Dv.data());
            for (int64_t i = 0; i < n; ++i) r[i] -= Dv[i];
        }
    return true;
}

// ------------------------------------------------------ even-odd --------
// Site parity (x + y + z + t) mod 2.  With every extent even, every hop joins
// sites of opposite parity, so D = [[A_ee, D_eo], [D_oe, A_oo]] and D phi = eta
// reduces to the Schur complement on the even sites:
//   Dhat = A_ee - D_eo A_oo^{-1} D_oe,
//   Dhat phi_e = eta_e - D_eo A_oo^{-1} eta_o,
//   phi_o = A_oo^{-1} (eta_o - D_oe phi_e).
int parity(const Lattice& lat, int64_t x) {
    int c[4];
    lat.coords(x, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

bool even_extents(const Lattice& lat) {
    for (int mu = 0; mu < 4; ++mu)
        if (lat.L[mu] % 2) return false;
    return true;
}

// out_p = A_pp^{-1} in_p at the sites of parity p (other sites left alone).
void site_inverse_apply(const Lattice& lat, double kappa, double csw, int p, const cplx* in, cplx* out) {
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < lat.V; ++x) {
        if (parity(lat, x) != p) continue;
        cplx A[144], Ai[144];
        site_term(lat, kappa, csw, x, A);
        invert(12, A, Ai);
        matvec12(Ai, in + x * 12, out + x * 12);
    }
}

// out_p = (hopping part of D) in, at the sites of parity p, reading only the
// opposite parity of in; other sites of out left alone.
void hops_parity(const Lattice& lat, double kappa, int p, const cplx* in, cplx* out) {
    Fetch other = [&lat, in, p](int64_t y) -> const cplx* { return parity(lat, y) != p ? in + y * 12 : nullptr; };
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < lat.V; ++x)
        if (parity(lat, x) == p) hops_at(lat, kappa, other, x, out + x * 12);
}

// out = Dhat psi on the even sites, 0 on the odd sites (psi's odd sites unused).
void apply_schur(const Lattice& lat, double kappa, double csw, const cplx* psi, cplx* out) {
    const int64_t n = lat.V * 12;
    std::vector<cplx> h(n, 0.0), t(n, 0.0), w(n, 0.0);
    hops_parity(lat, kappa, 1, psi, h.data());                 // D_oe psi_e
    site_inverse_apply(lat, kappa, csw, 1, h.data(), t.data());  // A_oo^{-1} D_oe psi_e
    hops_parity(lat, kappa, 0, t.data(), w.data());            // D_eo A_oo^{-1} D_oe psi_e
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < lat.V; ++x) {
        if (parity(lat, x) != 0) {
            for (int i = 0; i < 12; ++i) out[x * 12 + i] = 0.0;
            continue;
        }
        cplx A[144], a[12];
        site_term(lat, kappa, csw, x, A);
        matvec12(A, psi + x * 12, a);
        for (int i = 0; i < 12; ++i) out[x * 12 + i] = a[i] - w[x * 12 + i];
    }
}

thread_local char g_err[256] = "";

}  // namespace

// =============================================================== C ABI ===
extern "C" {

struct oracle_lattice {
    Lattice lat;
};

const char* oracle_last_error() { return g_err; }

// dims[4] = Lx,Ly,Lz,Lt; bc[4] = +-1; U = complex128 [V][4][3][3] (must stay
// alive while the handle is used); precompute_clover = 1 stores C(x) for all
// sites, 0 recomputes it on demand.
oracle_lattice* oracle_create(const int* dims, const int* bc, const double* U, int precompute_clover) {
    auto* h = new oracle_lattice;
    h->lat.V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        h->lat.L[mu] = dims[mu];
        h->lat.bc[mu] = bc ? bc[mu] : 1;
        h->lat.V *= dims[mu];
    }
    h->lat.U = reinterpret_cast<const cplx*>(U);
    if (precompute_clover) {
        h->lat.clover.assign(h->lat.V * 144, 0.0);
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < h->lat.V; ++x) clover_site(h->lat, x, h->lat.clover.data() + x * 144);
    }
    return h;
}

void oracle_destroy(oracle_lattice* h) { delete h; }

int oracle_num_threads() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// Number of OpenMP threads for the following calls (timing at 1 thread and at
// all cores).
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

// gamma matrices [4][4][4] complex and sigma [4][4][4][4] complex, for tests.
void oracle_gammas(double* g, double* sigma) {
    std::memcpy(g, DIRAC.g, sizeof(DIRAC.g));
    std::memcpy(sigma, DIRAC.sigma, sizeof(DIRAC.sigma));
}

// C(x) as [n][12][12] complex for the given sites.
void oracle_clover(oracle_lattice* h, int64_t n, const int64_t* sites, double* out) {
    cplx* o = reinterpret_cast<cplx*>(out);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        cplx tmp[144];
        const cplx* C = clover_of(h->lat, sites[k], tmp);
        std::memcpy(o + k * 144, C, sizeof(tmp));
    }
}

// out = D psi on the whole lattice; psi, out complex128 [V][4][3].
void oracle_apply_D(oracle_lattice* h, double kappa, double csw, const double* psi, double* out) {
    apply_D(h->lat, kappa, csw, reinterpret_cast<const cplx*>(psi), reinterpret_cast<cplx*>(out));
}

// (D psi)(x) at n listed sites only; out complex128 [n][4][3].
void oracle_apply_D_sites(oracle_lattice* h, double kappa, double csw, const double* psi, int64_t n,
                          const int64_t* sites, double* out) {
    const cplx* p = reinterpret_cast<const cplx*>(psi);
    cplx* o = reinterpret_cast<cplx*>(out);
    Fetch whole = [p](int64_t y) { return p + y * 12; };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) D_at(h->lat, kappa, csw, whole, sites[k], o + k * 12);
}

// Number of blocks and extended-block volume for block shape b and overlap s;
// returns 0 on success, -1 if the shape does not tile the lattice.
int oracle_decomp(oracle_lattice* h, const int* b, int s, int64_t* nblocks, int64_t* ext_volume) {
    Decomp d;
    if (!make_decomp(h->lat, b, s, &d)) {
        std::snprintf(g_err, sizeof g_err, "block shape does not tile the lattice");
        return -1;
    }
    *nblocks = d.nblocks;
    *ext_volume = d.ext_volume;
    return 0;
}

// Global site indices of Omega'_blk in local lexicographic order.
int oracle_block_sites(oracle_lattice* h, const int* b, int s, int64_t blk, int64_t* sites) {
    Decomp d;
    if (!make_decomp(h->lat, b, s, &d) || blk < 0 || blk >= d.nblocks) return -1;
    std::vector<int64_t> v = ext_sites(h->lat, d, blk);
    std::copy(v.begin(), v.end(), sites);
    return 0;
}

// out = D_{Omega'_blk} in, both complex128 [ext_volume][4][3] in the order of
// oracle_block_sites.
int oracle_block_apply(oracle_lattice* h, const int* b, int s, int64_t blk, double kappa, double csw,
                       const double* in, double* out) {
    Decomp d;
    if (!make_decomp(h->lat, b, s, &d) || blk < 0 || blk >= d.nblocks) return -1;
    BlockOp op(h->lat, d, blk);
    const std::vector<int64_t>& sites = op.sites;
    const cplx* pin = reinterpret_cast<const cplx*>(in);
    std::vector<cplx> vin(pin, pin + sites.size() * 12), vout(sites.size() * 12);
    op.apply(kappa, csw, vin, vout);
    std::memcpy(out, vout.data(), vout.size() * sizeof(cplx));
    return 0;
}

// x = MR^n applied to rhs on block blk (zero start, n steps).
int oracle_block_mr(oracle_lattice* h, const int* b, int s, int64_t blk, double kappa, double csw,
                    int n, const double* rhs, double* x) {
    Decomp d;
    if (!make_decomp(h->lat, b, s, &d) || blk < 0 || blk >= d.nblocks) return -1;
    BlockOp op(h->lat, d, blk);
    const std::vector<int64_t>& sites = op.sites;
    const cplx* pr = reinterpret_cast<const cplx*>(rhs);
    std::vector<cplx> vb(pr, pr + sites.size() * 12), vx;
    mr_solve(op, kappa, csw, vb, vx, n);
    std::memcpy(x, vx.data(), vx.size() * sizeof(cplx));
    return 0;
}

// phi = K eta for the Schwarz iteration `schwarz` (0 = RAS, Algorithm 1;
// 1 = additive; 2 = multiplicative) with domain solver `solver` (0 = MR,
// 1 = block Jacobi, 2 = truncated BiCGStab). exact = 1 solves each domain to
// 1e-14 instead.
int oracle_schwarz(oracle_lattice* h, const int* b, int s, int n_ras, int n_dominv, int exact, int solver,
                   int schwarz, double kappa, double csw, const double* eta, double* phi) {
    RasParams P;
    for (int mu = 0; mu < 4; ++mu) P.b[mu] = b[mu];
    P.s = s;
    P.n_ras = n_ras;
    P.n_dominv = n_dominv;
    P.exact = exact;
    P.solver = solver;
    P.schwarz = schwarz;
    const int64_t n = h->lat.V * 12;
    const cplx* pe = reinterpret_cast<const cplx*>(eta);
    std::vector<cplx> e(pe, pe + n), f;
    if (!ras(h->lat, P, kappa, csw, e, f)) {
        std::snprintf(g_err, sizeof g_err, "block shape does not tile the lattice");
        return -1;
    }
    std::memcpy(phi, f.data(), n * sizeof(cplx));
    return 0;
}

// x = n iterations of domain solver `solver` (as oracle_schwarz) on block blk
// from zero, right-hand side rhs (ext_volume sites, oracle_block_sites order).
int oracle_block_solve(oracle_lattice* h, const int* b, int s, int64_t blk, double kappa, double csw, int solver,
                       int n, const double* rhs, double* x) {
    Decomp d;
    if (!make_decomp(h->lat, b, s, &d) || blk < 0 || blk >= d.nblocks || solver < 0 || solver > 2) return -1;
    BlockOp op(h->lat, d, blk);
    const cplx* pr = reinterpret_cast<const cplx*>(rhs);
    std::vector<cplx> vb(pr, pr + op.sites.size() * 12), vx;
    if (solver == DOM_JACOBI) jacobi_solve(op, kappa, csw, vb, vx, n);
    else if (solver == DOM_BICGSTAB) bicgstab_fixed(op, kappa, csw, vb, vx, n);
    else mr_solve(op, kappa, csw, vb, vx, n);
    std::memcpy(x, vx.data(), vx.size() * sizeof(cplx));
    return 0;
}

// A(x)^{-1} = (1 + c_sw kappa C(x))^{-1} as [n][12][12] complex at the listed
// sites; -1 if some A(x) is singular.
int oracle_site_term_inverse(oracle_lattice* h, double kappa, double csw, int64_t n, const int64_t* sites,
                             double* out) {
    cplx* o = reinterpret_cast<cplx*>(out);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t k = 0; k < n; ++k) {
        cplx A[144];
        site_term(h->lat, kappa, csw, sites[k], A);
        if (!invert(12, A, o + k * 144)) ++bad;
    }
    return bad ? -1 : 0;
}

// phi = K_RAS eta (Algorithm 1). exact = 1 solves each domain to 1e-14.
int oracle_ras(oracle_lattice* h, const int* b, int s, int n_ras, int n_dominv, int exact, double kappa,
               double csw, const double* eta, double* phi) {
    RasParams P;
    for (int mu = 0; mu < 4; ++mu) P.b[mu] = b[mu];
    P.s = s;
    P.n_ras = n_ras;
    P.n_dominv = n_dominv;
    P.exact = exact;
    P.solver = DOM_MR;
    P.schwarz = SCH_RAS;
    const int64_t n = h->lat.V * 12;
    const cplx* pe = reinterpret_cast<const cplx*>(eta);
    std::vector<cplx> e(pe, pe + n), f;
    if (!ras(h->lat, P, kappa, csw, e, f)) {
        std::snprintf(g_err, sizeof g_err, "block shape does not tile the lattice");
        return -1;
    }
    std::memcpy(phi, f.data(), n * sizeof(cplx));
    return 0;
}

// out = Dhat psi (the even-odd Schur complement on the even sites, 0 on the
// odd sites); -1 if an extent is odd.
int oracle_apply_schur(oracle_lattice* h, double kappa, double csw, const double* psi, double* out) {
    if (!even_extents(h->lat)) {
        std::snprintf(g_err, sizeof g_err, "even-odd reduction needs even extents");
        return -1;
    }
    apply_schur(h->lat, kappa, csw, reinterpret_cast<const cplx*>(psi), reinterpret_cast<cplx*>(out));
    return 0;
}

// D phi = eta through the even-odd reduction: BiCGStab (tolerance tol on
// the reduced system's recursive residual) on Dhat phi_e = eta_e - D_eo
// A_oo^{-1} eta_o, then phi_o = A_oo^{-1}(eta_o - D_oe phi_e).
// info = {iterations, restarts, converged}.
int oracle_eo_solve(oracle_lattice* h, double kappa, double csw, double tol, int max_iter, const double* eta,
                    double* phi, int* info, double* rel_resid) {
    const Lattice& lat = h->lat;
    if (!even_extents(lat)) {
        std::snprintf(g_err, sizeof g_err, "even-odd reduction needs even extents");
        return -1;
    }
    const int64_t n = lat.V * 12;
    const cplx* pe = reinterpret_cast<const cplx*>(eta);
    std::vector<cplx> t(n, 0.0), w(n, 0.0), be(n, 0.0), x;
    site_inverse_apply(lat, kappa, csw, 1, pe, t.data());   // A_oo^{-1} eta_o
    hops_parity(lat, kappa, 0, t.data(), w.data());         // D_eo A_oo^{-1} eta_o
    for (int64_t y = 0; y < lat.V; ++y)
        if (parity(lat, y) == 0)
            for (int i = 0; i < 12; ++i) be[y * 12 + i] = pe[y * 12 + i] - w[y * 12 + i];
    VecOp A = [&](const std::vector<cplx>& a, std::vector<cplx>& o) {
        o.resize(a.size());
        apply_schur(lat, kappa, csw, a.data(), o.data());
    };
    SolveInfo si = bicgstab(A, nullptr, be, x, tol, max_iter);
    // odd sites: phi_o = A_oo^{-1}(eta_o - D_oe phi_e)
    std::vector<cplx> hx(n, 0.0), ro(n, 0.0);
    hops_parity(lat, kappa, 1, x.data(), hx.data());
    for (int64_t y = 0; y < lat.V; ++y)
        if (parity(lat, y) == 1)
            for (int i = 0; i < 12; ++i) ro[y * 12 + i] = pe[y * 12 + i] - hx[y * 12 + i];
    site_inverse_apply(lat, kappa, csw, 1, ro.data(), x.data());
    std::memcpy(phi, x.data(), n * sizeof(cplx));
    info[0] = si.iters;
    info[1] = si.restarts;
    info[2] = si.converged;
    *rel_resid = si.rel_resid;
    return si.converged ? 0 : 1;
}

// Plain BiCGStab on D phi = eta; info = {iterations, restarts, converged}
// and *rel_resid = recursive residual / |eta|.
int oracle_bicgstab(oracle_lattice* h, double kappa, double csw, double tol, int max_iter, const double* eta,
                    double* phi, int* info, double* rel_resid) {
    const int64_t n = h->lat.V * 12;
    const cplx* pe = reinterpret_cast<const cplx*>(eta);
    std::vector<cplx> b(pe, pe + n), x;
    VecOp A = [&](const std::vector<cplx>& a, std::vector<cplx>& o) {
        o.resize(a.size());
        apply_D(h->lat, kappa, csw, a.data(), o.data());
    };
    SolveInfo si = bicgstab(A, nullptr, b, x, tol, max_iter);
    std::memcpy(phi, x.data(), n * sizeof(cplx));
    info[0] = si.iters;
    info[1] = si.restarts;
    info[2] = si.converged;
    *rel_resid = si.rel_resid;
    return si.converged ? 0 : 1;
}

// Nested BiCGStab (Sec. 3), both levels in FP64: the outer BiCGStab on
// D phi = eta uses as its preconditioner an inner BiCGStab that is itself
// right-preconditioned by K_RAS (Eq. (3)) and stops at tol_inner (or
// max_inner iterations).  use_ras = 0 drops K_RAS from the inner solver.
// info = {outer iterations, total inner iterations, converged}.
int oracle_nested(oracle_lattice* h, double kappa, double csw, double tol, int max_outer, double tol_inner,
                  int max_inner, int use_ras, const int* b, int s, int n_ras, int n_dominv, const double* eta,
                  double* phi, int* info, double* rel_resid) {
    const int64_t n = h->lat.V * 12;
    RasParams P;
    for (int mu = 0; mu < 4; ++mu) P.b[mu] = b[mu];
    P.s = s;
    P.n_ras = n_ras;
    P.n_dominv = n_dominv;
    P.exact = 0;
    P.solver = DOM_MR;
    P.schwarz = SCH_RAS;
    Decomp d;
    if (use_ras && !make_decomp(h->lat, P.b, P.s, &d)) {
        std::snprintf(g_err, sizeof g_err, "block shape does not tile the lattice");
        return -1;
    }
    VecOp A = [&](const std::vector<cplx>& a, std::vector<cplx>& o) {
        o.resize(a.size());
        apply_D(h->lat, kappa, csw, a.data(), o.data());
    };
    VecOp Kras = [&](const std::vector<cplx>& a, std::vector<cplx>& o) { ras(h->lat, P, kappa, csw, a, o); };
    int inner_total = 0;
    VecOp Kinner = [&](const std::vector<cplx>& a, std::vector<cplx>& o) {
        SolveInfo si = bicgstab(A, use_ras ? &Kras : nullptr, a, o, tol_inner, max_inner);
        inner_total += si.iters;
    };
    const cplx* pe = reinterpret_cast<const cplx*>(eta);
    std::vector<cplx> bvec(pe, pe + n), x;
    SolveInfo si = bicgstab(A, &Kinner, bvec, x, tol, max_outer);
    std::memcpy(phi, x.data(), n * sizeof(cplx));
    info[0] = si.iters;
    info[1] = inner_total;
    info[2] = si.converged;
    *rel_resid = si.rel_resid;
    return si.converged ? 0 : 1;
}

}  // extern "C"
