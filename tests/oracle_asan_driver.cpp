// Host sanitizer run of the FP64 oracle: built by tests/test_oracle_asan.py
// together with oracle/wcl_oracle.cpp under AddressSanitizer and
// UndefinedBehaviorSanitizer (g++ only, no device code), it drives every
// entry point of the oracle on small lattices, including odd extents, overlap
// 2, domains spanning whole directions and the extent-2 double hops, so that
// an out-of-bounds index or an undefined operation anywhere in the oracle
// aborts the run.  Prints "ok" and exits 0 when every call returned.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

extern "C" {
struct oracle_lattice;
oracle_lattice* oracle_create(const int* dims, const int* bc, const double* U, int precompute_clover);
void oracle_destroy(oracle_lattice* h);
void oracle_set_threads(int n);
void oracle_apply_D(oracle_lattice* h, double kappa, double csw, const double* psi, double* out);
void oracle_apply_D_sites(oracle_lattice* h, double kappa, double csw, const double* psi, int64_t n,
                          const int64_t* sites, double* out);
void oracle_clover(oracle_lattice* h, int64_t n, const int64_t* sites, double* out);
int oracle_decomp(oracle_lattice* h, const int* b, int s, int64_t* nblocks, int64_t* ext_volume);
int oracle_block_sites(oracle_lattice* h, const int* b, int s, int64_t blk, int64_t* sites);
int oracle_block_apply(oracle_lattice* h, const int* b, int s, int64_t blk, double kappa, double csw,
                       const double* in, double* out);
int oracle_block_mr(oracle_lattice* h, const int* b, int s, int64_t blk, double kappa, double csw, int n,
                    const double* rhs, double* x);
int oracle_schwarz(oracle_lattice* h, const int* b, int s, int n_ras, int n_dominv, int exact, int solver,
                   int schwarz, double kappa, double csw, const double* eta, double* phi);
int oracle_block_solve(oracle_lattice* h, const int* b, int s, int64_t blk, double kappa, double csw, int solver,
                       int n, const double* rhs, double* x);
int oracle_site_term_inverse(oracle_lattice* h, double kappa, double csw, int64_t n, const int64_t* sites,
                             double* out);
int oracle_apply_schur(oracle_lattice* h, double kappa, double csw, const double* psi, double* out);
int oracle_eo_solve(oracle_lattice* h, double kappa, double csw, double tol, int max_iter, const double* eta,
                    double* phi, int* info, double* rel_resid);
int oracle_bicgstab(oracle_lattice* h, double kappa, double csw, double tol, int max_iter, const double* eta,
                    double* phi, int* info, double* rel_resid);
int oracle_nested(oracle_lattice* h, double kappa, double csw, double tol, int max_outer, double tol_inner,
                  int max_inner, int use_ras, const int* b, int s, int n_ras, int n_dominv, const double* eta,
                  double* phi, int* info, double* rel_resid);
}

using cplx = std::complex<double>;

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);   \
            std::exit(1);                                             \
        }                                                             \
    } while (0)

// Random SU(3) links: rows 0 and 1 orthonormalised from Gaussian rows, row 2
// = conj(row0 x row1) (unit determinant).
static std::vector<cplx> random_links(int64_t V, std::mt19937_64& rng) {
    std::normal_distribution<double> g;
    std::vector<cplx> U(V * 4 * 9);
    for (int64_t k = 0; k < V * 4; ++k) {
        cplx* u = &U[k * 9];
        for (int j = 0; j < 6; ++j) u[j] = cplx(g(rng), g(rng));
        double n0 = 0;
        for (int j = 0; j < 3; ++j) n0 += std::norm(u[j]);
        for (int j = 0; j < 3; ++j) u[j] /= std::sqrt(n0);
        cplx d = 0;
        for (int j = 0; j < 3; ++j) d += std::conj(u[j]) * u[3 + j];
        for (int j = 0; j < 3; ++j) u[3 + j] -= d * u[j];
        double n1 = 0;
        for (int j = 0; j < 3; ++j) n1 += std::norm(u[3 + j]);
        for (int j = 0; j < 3; ++j) u[3 + j] /= std::sqrt(n1);
        for (int c = 0; c < 3; ++c) {
            const int a = (c + 1) % 3, b = (c + 2) % 3;
            u[6 + c] = std::conj(u[a] * u[3 + b] - u[b] * u[3 + a]);
        }
    }
    return U;
}

static std::vector<cplx> random_field(int64_t V, std::mt19937_64& rng) {
    std::normal_distribution<double> g;
    std::vector<cplx> v(V * 12);
    for (auto& z : v) z = cplx(g(rng), g(rng));
    return v;
}

static const double* D(const std::vector<cplx>& v) { return reinterpret_cast<const double*>(v.data()); }
static double* D(std::vector<cplx>& v) { return reinterpret_cast<double*>(v.data()); }

struct Case {
    int dims[4];
    int bc[4];
    int b[4];
    int s;
};

int main() {
    oracle_set_threads(2);
    std::mt19937_64 rng(7);
    const Case cases[] = {
        {{4, 4, 4, 4}, {1, 1, 1, 1}, {2, 2, 2, 2}, 1},
        {{6, 4, 2, 4}, {1, 1, 1, -1}, {3, 2, 2, 2}, 0},    // extent 2: forward = backward neighbour
        {{8, 4, 4, 4}, {1, 1, 1, 1}, {2, 4, 4, 4}, 2},     // x-only split, overlap 2
        {{5, 3, 4, 2}, {1, -1, 1, 1}, {5, 3, 2, 2}, 1},    // odd extents, domains spanning x and y
    };
    const double kappa = 0.123, csw = 1.2;
    for (const Case& c : cases) {
        const int64_t V = (int64_t)c.dims[0] * c.dims[1] * c.dims[2] * c.dims[3];
        std::vector<cplx> U = random_links(V, rng);
        for (int pre = 0; pre < 2; ++pre) {
            oracle_lattice* h = oracle_create(c.dims, c.bc, D(U), pre);
            std::vector<cplx> psi = random_field(V, rng), out(V * 12), phi(V * 12);
            oracle_apply_D(h, kappa, csw, D(psi), D(out));
            std::vector<int64_t> sites = {0, V - 1, V / 2};
            std::vector<cplx> part(sites.size() * 12), cl(sites.size() * 144), ai(sites.size() * 144);
            oracle_apply_D_sites(h, kappa, csw, D(psi), (int64_t)sites.size(), sites.data(), D(part));
            oracle_clover(h, (int64_t)sites.size(), sites.data(), D(cl));
            CHECK(oracle_site_term_inverse(h, kappa, csw, (int64_t)sites.size(), sites.data(), D(ai)) == 0);
            int64_t nb = 0, ev = 0;
            CHECK(oracle_decomp(h, c.b, c.s, &nb, &ev) == 0);
            std::vector<int64_t> es(ev);
            std::vector<cplx> bin = random_field(ev, rng), bout(ev * 12);
            for (int64_t blk = 0; blk < nb; blk += (nb > 3 ? nb / 3 : 1)) {
                CHECK(oracle_block_sites(h, c.b, c.s, blk, es.data()) == 0);
                CHECK(oracle_block_apply(h, c.b, c.s, blk, kappa, csw, D(bin), D(bout)) == 0);
                CHECK(oracle_block_mr(h, c.b, c.s, blk, kappa, csw, 3, D(bin), D(bout)) == 0);
                for (int sv = 0; sv < 3; ++sv)
                    CHECK(oracle_block_solve(h, c.b, c.s, blk, kappa, csw, sv, 3, D(bin), D(bout)) == 0);
            }
            for (int sv = 0; sv < 3; ++sv)
                for (int sz = 0; sz < 3; ++sz)
                    CHECK(oracle_schwarz(h, c.b, c.s, 2, 2, 0, sv, sz, kappa, csw, D(psi), D(phi)) == 0);
            CHECK(oracle_schwarz(h, c.b, c.s, 1, 1, 1, 0, 0, kappa, csw, D(psi), D(phi)) == 0);
            int info[3];
            double rel = 0;
            oracle_bicgstab(h, kappa, csw, 1e-8, 200, D(psi), D(phi), info, &rel);
            oracle_nested(h, kappa, csw, 1e-8, 20, 1e-3, 20, 1, c.b, c.s, 2, 2, D(psi), D(phi), info, &rel);
            const bool even = c.dims[0] % 2 == 0 && c.dims[1] % 2 == 0 && c.dims[2] % 2 == 0 && c.dims[3] % 2 == 0;
            CHECK((oracle_apply_schur(h, kappa, csw, D(psi), D(out)) == 0) == even);
            if (even) CHECK(oracle_eo_solve(h, kappa, csw, 1e-8, 200, D(psi), D(phi), info, &rel) >= 0);
            // a block shape that does not tile the lattice is an error, not a fault
            const int bad[4] = {c.dims[0] + 1, 1, 1, 1};
            CHECK(oracle_decomp(h, bad, 0, &nb, &ev) != 0);
            oracle_destroy(h);
        }
    }
    std::printf("ok\n");
    return 0;
}
