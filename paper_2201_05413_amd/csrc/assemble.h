// assemble.h -- host assembly of the library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "femcg.h"

namespace femcg {

// Allocator that leaves trivially constructible elements uninitialised, so
// that a large array is first touched (and paged in) by the parallel loop
// that fills every element, not by one thread zeroing it first.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <typename U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept
    {
    }
    template <typename U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value)
    {
        ::new ((void *)p) U;
    }
    template <typename U, typename... Args>
    void construct(U *p, Args &&...args)
    {
        ::new ((void *)p) U(std::forward<Args>(args)...);
    }
};
template <typename T>
using BigVec = std::vector<T, NoInitAlloc<T>>;

struct HostSystem {
    int dim = 0, order = 0, nloc = 0;
    int64_t nverts = 0, ncells = 0, nedges = 0, ndofs = 0, nfree = 0, ndir = 0;
    std::vector<double> dof_coords;      // [ndofs][dim]
    std::vector<uint8_t> dirichlet;      // [ndofs]
    std::vector<int64_t> free2dof, dof2free, dir2dof, dof2dir;
    std::vector<int32_t> cell_dofs;      // [ncells][nloc] (released after assembly)
    // A = K_II, structural pattern, columns ascending (free numbering)
    std::vector<int64_t> a_rowptr;
    BigVec<int32_t> a_col;
    BigVec<double> a_val;
    // K_ID: free rows x Dirichlet columns (Dirichlet numbering)
    std::vector<int64_t> l_rowptr;
    BigVec<int32_t> l_col;
    BigVec<double> l_val;
};

// Solver copy of A on the host, in internal (permuted) row order.
struct SolverCopy {
    int format = FEM_FORMAT_CSR, C = 64, sigma = 1, sfc = 0;
    int64_t n = 0, nnz = 0, stored = 0;
    std::vector<int32_t> perm;           // internal row -> free row
    std::vector<double> diag;            // free order
    std::vector<int32_t> rowptr;         // internal CSR
    BigVec<int32_t> col;
    BigVec<double> val;
    std::vector<double> dinv;            // internal order
    std::vector<int64_t> slice_ptr;      // SELL
    std::vector<int32_t> rowlen;
    BigVec<int32_t> sell_col;
    BigVec<double> sell_val;
};

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn);
int assemble_host(const fem_mesh *mesh, int order, HostSystem &hs, std::string &err);
// Same result computed on the device (stream s): edges, boundary facets,
// element matrices, and the (row, col) sort and run sums of the element
// entries; the host system is filled from the device results.  Returns
// FEMCG_EUNSUPPORTED for meshes beyond its index ranges (callers then use
// assemble_host).
int assemble_device(const fem_mesh *mesh, int order, HostSystem &hs, std::string &err, hipStream_t s);
// P3/P4 triangles: the geometry-free table M^{mn}_{ij} = (1/|T|) integral
// (d phi_i / d l_m)(d phi_j / d l_n), [3][3][nl][nl], local DOFs: vertices,
// then the p-1 points of edges (0,1), (0,2), (1,2) from their first vertex on,
// then interior points in decreasing lexicographic order.
const std::vector<double> &pk_moment_table(int k, int *nl);
int build_solver_copy(const HostSystem &hs, int format, int C, int sigma, SolverCopy &sc,
                      std::string &err, int sfc = 0);

}  // namespace femcg
