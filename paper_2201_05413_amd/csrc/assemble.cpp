// assemble.cpp -- host-side FEM assembly of the library (mesh -> A = K_II,
// lifting operator K_ID, solver copy).
//
// The stiffness matrix is K_ij = integral grad(phi_i).grad(phi_j) for the P1
// or P2 Lagrange basis: the sign-flipped, symmetric counterpart of the
// paper's Laplacian matrix (Sect. 2.2: off-diagonal cotangent weights w(i,j),
// diagonal -sum_j w(i,j)).  Element matrices use the closed-form simplex
// moments  integral l^a = |T| d! a! / (d + |a|)!  of the barycentric
// coordinates l, so no quadrature is involved:
//   integral l_a       = |T| / (d+1)
//   integral l_a l_b   = |T| (1 + [a=b]) / ((d+1)(d+2))
// With g_a = grad l_a, the P2 basis is l_a(2 l_a - 1) at vertices and
// 4 l_a l_b at edges, whose gradients are (4 l_a - 1) g_a and
// 4 (l_a g_b + l_b g_a); products of these integrate with the moments above.
//
// P3 and P4 triangles (Table 7's degrees 3 and 4) use the product form of
// the Lagrange basis on the equispaced lattice (Silvester): for a lattice
// point with barycentric index (a_0, a_1, a_2), a_0 + a_1 + a_2 = k,
//   phi = prod_m R_{a_m}(l_m),   R_a(t) = prod_{s<a} (k t - s) / (s + 1),
// so grad phi = sum_m (d phi / d l_m) g_m and
//   K = |T| sum_{m,n} (g_m . g_n) M^{mn},
//   M^{mn}_{ij} = (1/|T|) integral (d phi_i / d l_m)(d phi_j / d l_n),
// a geometry-free table built once per degree from the 2D moments
//   integral l_0^a l_1^b l_2^c = 2 |T| a! b! c! / (a + b + c + 2)!.
//
// Dirichlet lifting with zero source (Sect. 2.2, u = f on the boundary;
// b encodes the boundary condition): A = K_II, b = -K_ID g_D.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "assemble.h"
#include "element.h"

namespace femcg {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn)
{
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
    if (n < 4096 || nt <= 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([&fn, b, e] { fn(b, e); });
    }
    for (auto &x : th) x.join();
}

// ---- P3 / P4 triangles ----------------------------------------------------

// Local numbering of a degree-k triangle: the three vertices, then the k-1
// points of each edge (0,1), (0,2), (1,2) from its first vertex on, then the
// interior points in decreasing lexicographic order of their index.
static int pk_local_index(int k, int idx[15][3])
{
    int c = 0;
    for (int v = 0; v < 3; ++v) {
        idx[c][0] = idx[c][1] = idx[c][2] = 0;
        idx[c++][v] = k;
    }
    const int ed[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto &e : ed)
        for (int s = 1; s < k; ++s) {
            idx[c][0] = idx[c][1] = idx[c][2] = 0;
            idx[c][e[0]] = k - s;
            idx[c++][e[1]] = s;
        }
    for (int a0 = k - 2; a0 >= 1; --a0)
        for (int a1 = k - 1 - a0; a1 >= 1; --a1) {
            idx[c][0] = a0;
            idx[c][1] = a1;
            idx[c++][2] = k - a0 - a1;
        }
    return c;
}

namespace {
struct PkTable {
    int k = 0, nl = 0;
    std::vector<double> M;  // [3][3][nl][nl]
};
}  // namespace

static const PkTable &pk_table(int k)
{
    static PkTable tab[5];
    static std::once_flag once[5];
    std::call_once(once[k], [k] {
        PkTable &T = tab[k];
        int idx[15][3];
        T.k = k;
        T.nl = pk_local_index(k, idx);
        const int nl = T.nl, D = k + 1;
        // R_a and R_a' as coefficient vectors in t (degree <= k)
        std::vector<std::vector<double>> R(k + 1, std::vector<double>(D, 0.0)), dR = R;
        for (int a = 0; a <= k; ++a) {
            std::vector<double> p(D, 0.0);
            p[0] = 1.0;
            for (int s0 = 0; s0 < a; ++s0) {  // p *= (k t - s0) / (s0 + 1)
                std::vector<double> q(D, 0.0);
                for (int e = 0; e < D; ++e) {
                    if (p[e] == 0.0) continue;
                    q[e] += -s0 * p[e] / (s0 + 1);
                    if (e + 1 < D) q[e + 1] += k * p[e] / (s0 + 1);
                }
                p = q;
            }
            R[a] = p;
            for (int e = 1; e < D; ++e) dR[a][e - 1] = e * p[e];
        }
        // d phi_i / d l_m as a dense coefficient cube over (e0, e1, e2)
        const int D3 = D * D * D;
        std::vector<double> dphi((size_t)nl * 3 * D3, 0.0);
        for (int i = 0; i < nl; ++i)
            for (int m = 0; m < 3; ++m) {
                double *c = &dphi[((size_t)i * 3 + m) * D3];
                const std::vector<double> *f[3];
                for (int r = 0; r < 3; ++r) f[r] = r == m ? &dR[idx[i][r]] : &R[idx[i][r]];
                for (int e0 = 0; e0 < D; ++e0)
                    for (int e1 = 0; e1 < D; ++e1)
                        for (int e2 = 0; e2 < D; ++e2)
                            c[(e0 * D + e1) * D + e2] = (*f[0])[e0] * (*f[1])[e1] * (*f[2])[e2];
            }
        double fact[2 * 5 + 3];
        fact[0] = 1.0;
        for (int i = 1; i < 13; ++i) fact[i] = fact[i - 1] * i;
        auto moment = [&](int a, int b, int c) { return 2.0 * fact[a] * fact[b] * fact[c] / fact[a + b + c + 2]; };
        T.M.assign((size_t)9 * nl * nl, 0.0);
        std::vector<int> nz;
        for (int i = 0; i < nl; ++i)
            for (int m = 0; m < 3; ++m)
                for (int j = 0; j < nl; ++j)
                    for (int n = 0; n < 3; ++n) {
                        const double *a = &dphi[((size_t)i * 3 + m) * D3], *b = &dphi[((size_t)j * 3 + n) * D3];
                        double sum = 0.0;
                        for (int x = 0; x < D3; ++x) {
                            if (a[x] == 0.0) continue;
                            const int x0 = x / (D * D), x1 = (x / D) % D, x2 = x % D;
                            for (int y = 0; y < D3; ++y) {
                                if (b[y] == 0.0) continue;
                                sum += a[x] * b[y] * moment(x0 + y / (D * D), x1 + (y / D) % D, x2 + y % D);
                            }
                        }
                        T.M[((size_t)(m * 3 + n) * nl + i) * nl + j] = sum;
                    }
    });
    return tab[k];
}

// The table M^{mn}_{ij} of degree k, [3][3][nl][nl] (for the device assembly).
const std::vector<double> &pk_moment_table(int k, int *nl)
{
    const PkTable &T = pk_table(k);
    *nl = T.nl;
    return T.M;
}

// K (nl x nl, local order of pk_local_index) of a degree-k triangle P[3][2].
static bool pk_element_matrix(int k, const double *P, double *K)
{
    double g[4][3] = {}, area;
    if (!simplex_grads(2, P, g, &area)) return false;
    const PkTable &T = pk_table(k);
    const int nl = T.nl;
    for (int i = 0; i < nl * nl; ++i) K[i] = 0.0;
    for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
            const double G = area * (g[m][0] * g[n][0] + g[m][1] * g[n][1]);
            const double *Mmn = &T.M[(size_t)(m * 3 + n) * nl * nl];
            for (int i = 0; i < nl * nl; ++i) K[i] += G * Mmn[i];
        }
    return true;
}

// Stable sort of v by cmp on up to 16 threads: chunks sorted in parallel,
// then merged pairwise (stable merges), level by level; the result is the
// unique stable order, the same as one std::stable_sort.
template <typename V, typename Cmp>
static void parallel_stable_sort(V &v, Cmp cmp)
{
    const int64_t n = (int64_t)v.size();
    unsigned hw = std::thread::hardware_concurrency();
    int T = (int)std::min<unsigned>(hw ? hw : 1, 16);
    if (n < (1 << 16) || T <= 1) {
        std::stable_sort(v.begin(), v.end(), cmp);
        return;
    }
    std::vector<int64_t> b(T + 1);
    for (int t = 0; t <= T; ++t) b[t] = n * t / T;
    auto run = [](int ntask, const std::function<void(int)> &fn) {
        std::vector<std::thread> th;
        for (int i = 0; i < ntask; ++i) th.emplace_back(fn, i);
        for (auto &x : th) x.join();
    };
    run(T, [&](int t) { std::stable_sort(v.begin() + b[t], v.begin() + b[t + 1], cmp); });
    for (int w = 1; w < T; w *= 2) {
        const int npair = (T + 2 * w - 1) / (2 * w);
        run(npair, [&](int p) {
            const int lo = 2 * w * p, mid = std::min(T, lo + w), hi = std::min(T, lo + 2 * w);
            if (mid < hi) std::inplace_merge(v.begin() + b[lo], v.begin() + b[mid], v.begin() + b[hi], cmp);
        });
    }
}

struct Face {
    int32_t v[3];
    bool operator<(const Face &o) const
    {
        return v[0] != o.v[0] ? v[0] < o.v[0] : (v[1] != o.v[1] ? v[1] < o.v[1] : v[2] < o.v[2]);
    }
    bool operator==(const Face &o) const { return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2]; }
};

int assemble_host(const fem_mesh *mesh, int order, HostSystem &hs, std::string &err)
{
    const int dim = mesh->dim;
    if ((dim != 2 && dim != 3) || order < 1 || order > 4 || (order > 2 && dim != 2)) {
        err = "unsupported dimension or order (P1/P2 on triangles and tetrahedra, P3/P4 on triangles)";
        return FEMCG_EUNSUPPORTED;
    }
    if (mesh->nverts <= 0 || mesh->ncells <= 0 || !mesh->coords || !mesh->cells || !mesh->on_boundary) {
        err = "empty mesh or NULL array";
        return FEMCG_EINVAL;
    }
    if (mesh->nverts >= (int64_t)1 << 30) {
        err = "too many vertices for int32 indices";
        return FEMCG_EUNSUPPORTED;
    }
    const int64_t nv = mesh->nverts, nc = mesh->ncells;
    const int nvl = dim + 1;
    for (int64_t i = 0; i < nc * nvl; ++i)
        if (mesh->cells[i] < 0 || mesh->cells[i] >= nv) {
            err = "cell vertex index out of range";
            return FEMCG_EMESH;
        }
    hs.dim = dim;
    hs.order = order;
    hs.nverts = nv;
    hs.ncells = nc;
    int E[6][2];
    const int nel = local_edges(dim, E);
    const int nl = order <= 2 ? (order == 1 ? nvl : nvl + nel) : (order + 1) * (order + 2) / 2;
    const int ke = order - 1, ci = (order - 1) * (order - 2) / 2;  // DOFs per edge, per cell interior
    hs.nloc = nl;

    // ---- DOFs: vertices, then k-1 per edge (edges in (min, max) order), then
    //      the cell interiors in cell order ----
    std::vector<uint64_t> ekey;
    std::vector<uint64_t> edges;
    if (order >= 2) {
        ekey.resize(nc * nel);
        for (int64_t c = 0; c < nc; ++c)
            for (int e = 0; e < nel; ++e) {
                uint64_t a = (uint64_t)mesh->cells[c * nvl + E[e][0]];
                uint64_t b = (uint64_t)mesh->cells[c * nvl + E[e][1]];
                if (a > b) std::swap(a, b);
                ekey[c * nel + e] = (a << 32) | b;
            }
        edges = ekey;
        parallel_stable_sort(edges, std::less<uint64_t>());
        edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    }
    hs.nedges = (int64_t)edges.size();
    hs.ndofs = nv + ke * hs.nedges + (int64_t)ci * nc;
    if (hs.ndofs >= (int64_t)1 << 31) {
        err = "too many DOFs for int32 indices";
        return FEMCG_EUNSUPPORTED;
    }
    hs.dof_coords.resize(hs.ndofs * dim);
    std::memcpy(hs.dof_coords.data(), mesh->coords, sizeof(double) * nv * dim);
    // edge DOF t (1..k-1) of edge (a, b), a < b: ((k - t) x_a + t x_b) / k
    for (int64_t e = 0; e < hs.nedges; ++e) {
        const int64_t a = (int64_t)(edges[e] >> 32), b = (int64_t)(edges[e] & 0xffffffffu);
        for (int r = 0; r < dim; ++r) {
            const double xa = mesh->coords[a * dim + r], xb = mesh->coords[b * dim + r];
            if (order == 2)
                hs.dof_coords[(nv + e) * dim + r] = 0.5 * (xa + xb);
            else
                for (int t = 1; t <= ke; ++t)
                    hs.dof_coords[(nv + ke * e + t - 1) * dim + r] = ((double)(order - t) * xa + (double)t * xb) / order;
        }
    }
    hs.cell_dofs.resize(nc * nl);
    int pidx[15][3];
    if (order >= 3) pk_local_index(order, pidx);
    const int64_t ibase = nv + ke * hs.nedges;
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            const int32_t *cv = mesh->cells + c * nvl;
            for (int i = 0; i < nvl; ++i) hs.cell_dofs[c * nl + i] = cv[i];
            if (order == 2)
                for (int e = 0; e < nel; ++e) {
                    auto it = std::lower_bound(edges.begin(), edges.end(), ekey[c * nel + e]);
                    hs.cell_dofs[c * nl + nvl + e] = (int32_t)(nv + (it - edges.begin()));
                }
            if (order >= 3) {
                for (int e = 0; e < 3; ++e) {
                    const int la = E[e][0], lb = E[e][1];
                    const int64_t idx = std::lower_bound(edges.begin(), edges.end(), ekey[c * nel + e]) - edges.begin();
                    for (int s = 1; s < order; ++s) {
                        // lattice weight of the larger global vertex
                        const int t = cv[la] > cv[lb] ? order - s : s;
                        hs.cell_dofs[c * nl + 3 + e * ke + (s - 1)] = (int32_t)(nv + ke * idx + t - 1);
                    }
                }
                for (int r = 0; r < ci; ++r) {
                    const int *a = pidx[3 + 3 * ke + r];
                    const int64_t d = ibase + (int64_t)ci * c + r;
                    hs.cell_dofs[c * nl + 3 + 3 * ke + r] = (int32_t)d;
                    for (int q = 0; q < dim; ++q)
                        hs.dof_coords[d * dim + q] = ((double)a[0] * mesh->coords[(int64_t)cv[0] * dim + q] +
                                                      (double)a[1] * mesh->coords[(int64_t)cv[1] * dim + q] +
                                                      (double)a[2] * mesh->coords[(int64_t)cv[2] * dim + q]) / order;
                }
            }
        }
    });

    // ---- Dirichlet DOFs ----
    hs.dirichlet.assign(hs.ndofs, 0);
    for (int64_t v = 0; v < nv; ++v) hs.dirichlet[v] = mesh->on_boundary[v] ? 1 : 0;
    if (order >= 2) {
        auto bnd = [&](uint64_t key) {
            return mesh->on_boundary[key >> 32] && mesh->on_boundary[key & 0xffffffffu];
        };
        if (dim == 2) {
            // boundary facets are the edges of exactly one triangle
            std::vector<uint64_t> all = ekey;
            parallel_stable_sort(all, std::less<uint64_t>());
            for (size_t i = 0; i < all.size();) {
                size_t j = i;
                while (j < all.size() && all[j] == all[i]) ++j;
                if (j - i == 1 && bnd(all[i])) {
                    const int64_t idx = std::lower_bound(edges.begin(), edges.end(), all[i]) - edges.begin();
                    for (int t = 0; t < ke; ++t) hs.dirichlet[nv + ke * idx + t] = 1;
                }
                i = j;
            }
        } else {
            std::vector<Face> faces(nc * 4);
            for (int64_t c = 0; c < nc; ++c)
                for (int o = 0; o < 4; ++o) {
                    Face f;
                    int q = 0;
                    for (int t = 0; t < 4; ++t)
                        if (t != o) f.v[q++] = mesh->cells[c * 4 + t];
                    std::sort(f.v, f.v + 3);
                    faces[c * 4 + o] = f;
                }
            parallel_stable_sort(faces, [](const Face &a, const Face &b) { return a < b; });
            for (size_t i = 0; i < faces.size();) {
                size_t j = i;
                while (j < faces.size() && faces[j] == faces[i]) ++j;
                if (j - i == 1) {
                    const int32_t *v = faces[i].v;
                    if (mesh->on_boundary[v[0]] && mesh->on_boundary[v[1]] && mesh->on_boundary[v[2]]) {
                        const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
                        for (auto &p : pr) {
                            const uint64_t key = ((uint64_t)v[p[0]] << 32) | (uint64_t)v[p[1]];
                            const int64_t idx = std::lower_bound(edges.begin(), edges.end(), key) - edges.begin();
                            hs.dirichlet[nv + idx] = 1;
                        }
                    }
                }
                i = j;
            }
        }
    }
    hs.dof2free.assign(hs.ndofs, -1);
    hs.dof2dir.assign(hs.ndofs, -1);
    hs.free2dof.clear();
    hs.dir2dof.clear();
    for (int64_t d = 0; d < hs.ndofs; ++d) {
        if (hs.dirichlet[d]) {
            hs.dof2dir[d] = (int64_t)hs.dir2dof.size();
            hs.dir2dof.push_back(d);
        } else {
            hs.dof2free[d] = (int64_t)hs.free2dof.size();
            hs.free2dof.push_back(d);
        }
    }
    hs.nfree = (int64_t)hs.free2dof.size();
    hs.ndir = (int64_t)hs.dir2dof.size();

    // ---- element matrices (parallel over cells) ----
    BigVec<double> Ke((size_t)nc * nl * nl);  // every entry written below (or the mesh is rejected)
    std::atomic<int64_t> bad{0};
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
        double P[12];
        for (int64_t c = c0; c < c1; ++c) {
            for (int i = 0; i < nvl; ++i)
                for (int r = 0; r < dim; ++r) P[i * dim + r] = mesh->coords[(int64_t)mesh->cells[c * nvl + i] * dim + r];
            const bool ok = order <= 2 ? element_matrix(dim, order, P, &Ke[(size_t)c * nl * nl])
                                       : pk_element_matrix(order, P, &Ke[(size_t)c * nl * nl]);
            if (!ok) bad.fetch_add(1);
        }
    });
    if (bad.load()) {
        err = "mesh has " + std::to_string(bad.load()) + " cells with non-positive measure";
        return FEMCG_EMESH;
    }

    // ---- DOF -> incident (cell, local index), cells ascending ----
    const int64_t nd = hs.ndofs;
    std::vector<int64_t> inc_ptr(nd + 1, 0);
    for (int64_t i = 0; i < nc * nl; ++i) inc_ptr[hs.cell_dofs[i] + 1]++;
    for (int64_t d = 0; d < nd; ++d) inc_ptr[d + 1] += inc_ptr[d];
    std::vector<int64_t> inc(nc * nl);
    {
        std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t i = 0; i < nc * nl; ++i) inc[fill[hs.cell_dofs[i]]++] = i;  // i = c*nl + a
    }

    // ---- rows of the free DOFs: pattern (all DOFs sharing a cell), values
    //      summed in cell order; split into A (free cols) and K_ID ----
    const int64_t nf = hs.nfree;
    std::vector<int64_t> a_cnt(nf + 1, 0), l_cnt(nf + 1, 0);
    std::vector<std::vector<int32_t>> dummy;
    // pass 1: pattern sizes
    parallel_for(nf, [&](int64_t f0, int64_t f1) {
        std::vector<int32_t> cols;
        for (int64_t f = f0; f < f1; ++f) {
            const int64_t d = hs.free2dof[f];
            cols.clear();
            for (int64_t t = inc_ptr[d]; t < inc_ptr[d + 1]; ++t) {
                const int64_t c = inc[t] / nl;
                for (int b = 0; b < nl; ++b) cols.push_back(hs.cell_dofs[c * nl + b]);
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            int64_t na = 0, nl_ = 0;
            for (int32_t cdof : cols) (hs.dirichlet[cdof] ? nl_ : na)++;
            a_cnt[f + 1] = na;
            l_cnt[f + 1] = nl_;
        }
    });
    for (int64_t f = 0; f < nf; ++f) {
        a_cnt[f + 1] += a_cnt[f];
        l_cnt[f + 1] += l_cnt[f];
    }
    hs.a_rowptr = a_cnt;
    hs.l_rowptr = l_cnt;
    // every entry is written by pass 2
    hs.a_col.clear();
    hs.a_val.clear();
    hs.l_col.clear();
    hs.l_val.clear();
    hs.a_col.resize(a_cnt[nf]);
    hs.a_val.resize(a_cnt[nf]);
    hs.l_col.resize(l_cnt[nf]);
    hs.l_val.resize(l_cnt[nf]);
    // pass 2: columns and values
    parallel_for(nf, [&](int64_t f0, int64_t f1) {
        std::vector<int32_t> cols;
        std::vector<double> vals;
        for (int64_t f = f0; f < f1; ++f) {
            const int64_t d = hs.free2dof[f];
            cols.clear();
            for (int64_t t = inc_ptr[d]; t < inc_ptr[d + 1]; ++t) {
                const int64_t c = inc[t] / nl;
                for (int b = 0; b < nl; ++b) cols.push_back(hs.cell_dofs[c * nl + b]);
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            vals.assign(cols.size(), 0.0);
            for (int64_t t = inc_ptr[d]; t < inc_ptr[d + 1]; ++t) {
                const int64_t c = inc[t] / nl, a = inc[t] % nl;
                const double *Kc = &Ke[(size_t)c * nl * nl + a * nl];
                for (int b = 0; b < nl; ++b) {
                    const int32_t cd = hs.cell_dofs[c * nl + b];
                    const size_t pos = std::lower_bound(cols.begin(), cols.end(), cd) - cols.begin();
                    vals[pos] += Kc[b];
                }
            }
            int64_t pa = hs.a_rowptr[f], pl = hs.l_rowptr[f];
            for (size_t i = 0; i < cols.size(); ++i) {
                const int32_t cd = cols[i];
                if (hs.dirichlet[cd]) {
                    hs.l_col[pl] = (int32_t)hs.dof2dir[cd];
                    hs.l_val[pl++] = vals[i];
                } else {
                    hs.a_col[pa] = (int32_t)hs.dof2free[cd];
                    hs.a_val[pa++] = vals[i];
                }
            }
        }
    });
    hs.cell_dofs.clear();
    hs.cell_dofs.shrink_to_fit();
    return FEMCG_OK;
}

// Solver copy: drop |a| <= 4 eps max_row|a| (never the diagonal), permute rows
// symmetrically so that rows sorted by length (within windows of sigma rows)
// share SELL slices.
// Morton key of a point: each coordinate quantised to `bits` bits over the
// bounding box, bits interleaved (x lowest).
static uint64_t morton_key(const double *x, int dim, const double *lo, const double *inv, int bits)
{
    uint64_t q[3] = {0, 0, 0};
    const uint64_t top = (1ull << bits) - 1;
    for (int r = 0; r < dim; ++r) {
        double t = (x[r] - lo[r]) * inv[r];
        uint64_t v = t <= 0 ? 0 : (uint64_t)(t * (double)top + 0.5);
        q[r] = v > top ? top : v;
    }
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int r = dim - 1; r >= 0; --r) key = (key << 1) | ((q[r] >> b) & 1u);
    return key;
}

int build_solver_copy(const HostSystem &hs, int format, int C, int sigma, SolverCopy &sc,
                      std::string &err, int sfc)
{
    const int64_t n = hs.nfree;
    sc.n = n;
    sc.format = format;
    sc.C = C;
    sc.sfc = sfc;
    sc.sigma = std::max(1, sigma);
    // pruned rows in free order
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> len(n);
    std::vector<uint8_t> keep(hs.a_col.size());
    sc.diag.assign(n, 0.0);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            double mx = 0.0;
            for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t) mx = std::max(mx, std::fabs(hs.a_val[t]));
            const double thr = 4.0 * 2.220446049250313e-16 * mx;
            int32_t c = 0;
            for (int64_t t = hs.a_rowptr[i]; t < hs.a_rowptr[i + 1]; ++t) {
                const bool diag = hs.a_col[t] == i;
                if (diag) sc.diag[i] = hs.a_val[t];
                keep[t] = diag || std::fabs(hs.a_val[t]) > thr;
                c += keep[t];
            }
            len[i] = c;
        }
    });
    for (int64_t i = 0; i < n; ++i)
        if (!(sc.diag[i] > 0.0)) {
            err = "non-positive diagonal in A";
            return FEMCG_EMESH;
        }
    // permutation: optional Morton order, then the sigma sort
    sc.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) sc.perm[i] = (int32_t)i;
    if (sfc) {
        const int dim = hs.dim;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, inv[3];
        for (int64_t i = 0; i < n; ++i)
            for (int r = 0; r < dim; ++r) {
                const double x = hs.dof_coords[hs.free2dof[i] * dim + r];
                lo[r] = std::min(lo[r], x);
                hi[r] = std::max(hi[r], x);
            }
        for (int r = 0; r < dim; ++r) inv[r] = hi[r] > lo[r] ? 1.0 / (hi[r] - lo[r]) : 0.0;
        const int bits = dim == 3 ? 21 : 31;
        std::vector<uint64_t> key(n);
        parallel_for(n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) key[i] = morton_key(&hs.dof_coords[hs.free2dof[i] * dim], dim, lo, inv, bits);
        });
        parallel_stable_sort(sc.perm, [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    }
    if (format == FEM_FORMAT_SELL && sc.sigma > 1) {
        const int64_t nw = (n + sc.sigma - 1) / sc.sigma;
        parallel_for(nw, [&](int64_t w0, int64_t w1) {
            for (int64_t wi = w0; wi < w1; ++wi) {
                const int64_t w = wi * sc.sigma, e = std::min(n, w + sc.sigma);
                std::stable_sort(sc.perm.begin() + w, sc.perm.begin() + e,
                                 [&](int32_t a, int32_t b) { return len[a] > len[b]; });
            }
        });
    }
    std::vector<int32_t> iperm(n);
    for (int64_t i = 0; i < n; ++i) iperm[sc.perm[i]] = (int32_t)i;
    // internal CSR (columns in internal numbering, ascending)
    sc.rowptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) sc.rowptr[i + 1] = sc.rowptr[i] + len[sc.perm[i]];
    const int64_t nnz = sc.rowptr[n];
    if (nnz >= ((int64_t)1 << 31)) {
        err = "too many nonzeros for int32 row pointers";
        return FEMCG_EUNSUPPORTED;
    }
    sc.nnz = nnz;
    sc.col.clear();
    sc.val.clear();
    sc.col.resize(nnz);  // every entry is written by the row loop below
    sc.val.resize(nnz);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t src = sc.perm[i];
            row.clear();
            for (int64_t t = hs.a_rowptr[src]; t < hs.a_rowptr[src + 1]; ++t)
                if (keep[t]) row.emplace_back(iperm[hs.a_col[t]], hs.a_val[t]);
            std::sort(row.begin(), row.end(), [](auto &a, auto &b) { return a.first < b.first; });
            int64_t p = sc.rowptr[i];
            for (auto &e : row) {
                sc.col[p] = e.first;
                sc.val[p++] = e.second;
            }
        }
    });
    sc.dinv.resize(n);
    for (int64_t i = 0; i < n; ++i) sc.dinv[i] = 1.0 / sc.diag[sc.perm[i]];
    // SELL-C-sigma: slice s holds rows [s*C, s*C+C), entry e of row r at
    // slice_ptr[s] + e*C + (r mod C); padding: column = own row, value 0
    if (format == FEM_FORMAT_SELL) {
        const int64_t ns = (n + C - 1) / C;
        sc.slice_ptr.assign(ns + 1, 0);
        sc.rowlen.resize(n);
        for (int64_t s = 0; s < ns; ++s) {
            int32_t mx = 0;
            for (int64_t r = s * C; r < std::min(n, s * C + C); ++r) {
                sc.rowlen[r] = (int32_t)(sc.rowptr[r + 1] - sc.rowptr[r]);
                mx = std::max(mx, sc.rowlen[r]);
            }
            sc.slice_ptr[s + 1] = sc.slice_ptr[s] + (int64_t)mx * C;
        }
        const int64_t stored = sc.slice_ptr[ns];
        sc.sell_col.clear();
        sc.sell_val.clear();
        sc.sell_col.resize(stored);  // every entry, padding included, is written below
        sc.sell_val.resize(stored);
        parallel_for(ns, [&](int64_t s0, int64_t s1) {
            for (int64_t s = s0; s < s1; ++s) {
                const int64_t base = sc.slice_ptr[s];
                const int64_t width = (sc.slice_ptr[s + 1] - base) / C;
                for (int64_t r = s * C; r < s * C + C; ++r) {
                    const int64_t lr = r - s * C;
                    const int64_t own = r < n ? r : n - 1;
                    for (int64_t e = 0; e < width; ++e) {
                        const int64_t dst = base + e * C + lr;
                        if (r < n && e < sc.rowlen[r]) {
                            sc.sell_col[dst] = sc.col[sc.rowptr[r] + e];
                            sc.sell_val[dst] = sc.val[sc.rowptr[r] + e];
                        } else {
                            sc.sell_col[dst] = (int32_t)own;
                            sc.sell_val[dst] = 0.0;
                        }
                    }
                }
            }
        });
        sc.stored = stored;
    } else {
        sc.stored = nnz;
    }
    return FEMCG_OK;
}

}  // namespace femcg
