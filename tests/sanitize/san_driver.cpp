// Sanitizer driver (test infrastructure, CPU only).  Built with g++ and
// -fsanitize=address,undefined together with the library's host assembly
// (assemble.cpp: assembly and the solver copy, whose large arrays are left
// uninitialised and filled by parallel loops and sorts) and the oracle
// (femoracle.c).  For one mesh file it
//   - assembles A = K_II on the host with the library, and builds the solver
//     copy in CSR (natural order) and SELL (C = 32, sigma = 64, Morton order);
//   - builds the oracle's system;
//   - checks the library's A against the oracle's A (pattern identical,
//     values within 1e-12 of the row's largest entry), the solver copies'
//     products against the library's A, and the oracle's PCG on two columns
//     against its own Eq. (2) residual.
// Any invalid access, use of uninitialised-but-unwritten memory that ASan
// detects, or undefined behaviour aborts the run; a failed check exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "assemble.h"

extern "C" {
void *orc_build(int dim, int64_t nverts, const double *coords, int64_t ncells, const int32_t *cells,
                const uint8_t *on_boundary, int order, int *err);
void orc_free(void *h);
void orc_sizes(const void *h, int64_t *sz);
void orc_copy_A(const void *h, int64_t *rowptr, int32_t *col, double *val);
int orc_rhs(const void *h, const double *g_all, int k, double *B);
int orc_relres(const void *h, const double *B, const double *X, int k, double *relres);
int orc_pcg(const void *h, const double *B, int k, double tol, int64_t max_iter, double *X, int64_t *iters,
            double *relres, int32_t *restarts);
void orc_copy_dofs(const void *h, double *coords, uint8_t *dirichlet, int64_t *free2dof);
}

static int fails = 0;
#define CHECK(c, ...)                              \
    do {                                           \
        if (!(c)) {                                \
            std::printf("FAIL: " __VA_ARGS__);     \
            std::printf("\n");                     \
            ++fails;                               \
        }                                          \
    } while (0)

template <typename T>
static bool read_vec(FILE *f, std::vector<T> &v, int64_t n)
{
    v.resize((size_t)n);
    return n == 0 || std::fread(v.data(), sizeof(T), (size_t)n, f) == (size_t)n;
}

// y = A x with A in the solver copy's CSR or SELL layout, rows internal
static void sc_apply(const femcg::SolverCopy &sc, const std::vector<double> &x_int, std::vector<double> &y_int)
{
    y_int.assign((size_t)sc.n, 0.0);
    for (int64_t i = 0; i < sc.n; ++i) {
        double acc = 0.0;
        if (sc.format == FEM_FORMAT_SELL) {
            const int64_t s = i / sc.C, l = i % sc.C;
            for (int32_t e = 0; e < sc.rowlen[i]; ++e) {
                const int64_t idx = sc.slice_ptr[s] + (int64_t)e * sc.C + l;
                acc += sc.sell_val[idx] * x_int[sc.sell_col[idx]];
            }
        } else {
            for (int32_t t = sc.rowptr[i]; t < sc.rowptr[i + 1]; ++t) acc += sc.val[t] * x_int[sc.col[t]];
        }
        y_int[i] = acc;
    }
}

int main(int argc, char **argv)
{
    if (argc < 3) {
        std::printf("usage: %s mesh.bin order\n", argv[0]);
        return 2;
    }
    const int order = std::atoi(argv[2]);
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[3];
    if (std::fread(hdr, 8, 3, f) != 3) return 2;
    const int dim = (int)hdr[0];
    const int64_t nv = hdr[1], nc = hdr[2];
    std::vector<double> coords;
    std::vector<int32_t> cells;
    std::vector<uint8_t> bnd;
    if (!read_vec(f, coords, nv * dim) || !read_vec(f, cells, nc * (dim + 1)) || !read_vec(f, bnd, nv)) return 2;
    std::fclose(f);

    fem_mesh mesh{};
    mesh.dim = dim;
    mesh.nverts = nv;
    mesh.coords = coords.data();
    mesh.ncells = nc;
    mesh.cells = cells.data();
    mesh.on_boundary = bnd.data();

    femcg::HostSystem hs;
    std::string err;
    int rc = femcg::assemble_host(&mesh, order, hs, err);
    CHECK(rc == 0, "assemble_host rc %d: %s", rc, err.c_str());
    if (rc) return 1;

    void *h = orc_build(dim, nv, coords.data(), nc, cells.data(), bnd.data(), order, &rc);
    CHECK(h != nullptr, "orc_build err %d", rc);
    if (!h) return 1;
    int64_t sz[6];
    orc_sizes(h, sz);
    const int64_t n = sz[2], nnz = sz[4];
    CHECK(n == hs.nfree, "nfree %lld vs %lld", (long long)n, (long long)hs.nfree);
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> col((size_t)std::max<int64_t>(nnz, 1));
    std::vector<double> val((size_t)std::max<int64_t>(nnz, 1));
    orc_copy_A(h, rp.data(), col.data(), val.data());
    CHECK((int64_t)hs.a_col.size() == nnz, "nnz %zu vs %lld", hs.a_col.size(), (long long)nnz);
    double worst = 0.0;
    for (int64_t i = 0; i < n && fails == 0; ++i) {
        CHECK(hs.a_rowptr[i + 1] == rp[i + 1], "row %lld extent", (long long)i);
        double mx = 0.0;
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) mx = std::fmax(mx, std::fabs(val[t]));
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            CHECK(hs.a_col[t] == col[t], "row %lld column", (long long)i);
            worst = std::fmax(worst, std::fabs(hs.a_val[t] - val[t]) / mx);
        }
    }
    CHECK(worst <= 1e-12, "assembly differs from the oracle by %.3e", worst);

    // solver copies: products against the assembled A
    std::vector<double> x(n), y(n, 0.0);
    for (int64_t i = 0; i < n; ++i) x[i] = std::sin(0.37 * (double)i + 1.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t) y[i] += hs.a_val[t] * x[hs.a_col[t]];
    const int fmts[2][4] = {{FEM_FORMAT_CSR, 64, 1, 0}, {FEM_FORMAT_SELL, 32, 64, 1}};
    for (const auto &fm : fmts) {
        femcg::SolverCopy sc;
        rc = femcg::build_solver_copy(hs, fm[0], fm[1], fm[2], sc, err, fm[3]);
        CHECK(rc == 0, "build_solver_copy rc %d: %s", rc, err.c_str());
        if (rc) continue;
        std::vector<double> xi(n), yi;
        for (int64_t i = 0; i < n; ++i) xi[i] = x[sc.perm[i]];
        sc_apply(sc, xi, yi);
        double ey = 0.0, ny = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            ey = std::fmax(ey, std::fabs(yi[i] - y[sc.perm[i]]));
            ny = std::fmax(ny, std::fabs(y[sc.perm[i]]));
        }
        CHECK(ey <= 1e-12 * std::fmax(ny, 1.0), "solver copy (format %d) product differs by %.3e", fm[0], ey);
        for (int64_t i = 0; i < n; ++i) CHECK(sc.dinv[i] > 0.0, "dinv[%lld] not positive", (long long)i);
    }

    // oracle: lifting, PCG, Eq. (2)
    const int64_t ndofs = sz[0];
    std::vector<double> dc((size_t)ndofs * dim), g((size_t)ndofs * 2);
    std::vector<uint8_t> dir((size_t)ndofs);
    std::vector<int64_t> f2d((size_t)n);
    orc_copy_dofs(h, dc.data(), dir.data(), f2d.data());
    for (int64_t i = 0; i < ndofs; ++i) {
        g[2 * i] = 1.0 + 2.0 * dc[i * dim] - 3.0 * dc[i * dim + 1];
        g[2 * i + 1] = dc[i * dim] * dc[i * dim] - dc[i * dim + 1] * dc[i * dim + 1];
    }
    std::vector<double> B((size_t)n * 2), X((size_t)n * 2), rel(2);
    std::vector<int64_t> its(2);
    std::vector<int32_t> rs(2);
    CHECK(orc_rhs(h, g.data(), 2, B.data()) == 0, "orc_rhs");
    rc = orc_pcg(h, B.data(), 2, 1e-10, 100000, X.data(), its.data(), rel.data(), rs.data());
    CHECK(rc == 0, "orc_pcg rc %d", rc);
    std::vector<double> rel2(2);
    CHECK(orc_relres(h, B.data(), X.data(), 2, rel2.data()) == 0, "orc_relres");
    // the PCG's true residual and orc_relres round differently (sqrt(rr)/|b|
    // against sqrt(rr/bb)): equal to within rounding
    for (int j = 0; j < 2; ++j)
        CHECK(rel2[j] <= 1e-10 && std::fabs(rel2[j] - rel[j]) <= 1e-12 * rel[j], "column %d residual %.3e / %.3e", j,
              rel2[j], rel[j]);
    orc_free(h);
    std::printf("%s: n %lld nnz %lld max assembly diff %.3e, %d failure(s)\n", argv[1], (long long)n,
                (long long)nnz, worst, fails);
    return fails ? 1 : 0;
}
