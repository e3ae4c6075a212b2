// element.h -- P1/P2 element stiffness matrices, shared by the host and the
// device assembly (closed-form simplex moments; see assemble.cpp).
#pragma once

#include <hip/hip_runtime.h>

namespace femcg {

// barycentric gradients g[a][r] and the measure |T| of one simplex
__host__ __device__ inline bool simplex_grads(int dim, const double *P, double g[4][3], double *meas)
{
    if (dim == 2) {
        const double x1 = P[2] - P[0], y1 = P[3] - P[1];
        const double x2 = P[4] - P[0], y2 = P[5] - P[1];
        const double det = x1 * y2 - x2 * y1;
        if (!(det > 0.0)) return false;
        // inverse of [[x1 x2][y1 y2]]: rows are grad l_1, grad l_2
        g[1][0] = y2 / det;
        g[1][1] = -x2 / det;
        g[2][0] = -y1 / det;
        g[2][1] = x1 / det;
        g[0][0] = -g[1][0] - g[2][0];
        g[0][1] = -g[1][1] - g[2][1];
        *meas = 0.5 * det;
        return true;
    }
    double e[3][3];
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) e[c][r] = P[(c + 1) * 3 + r] - P[r];
    // grad l_{c+1} = (e_{c+1} x e_{c+2}) / det  (cyclic), det = e1 . (e2 x e3)
    double cr[3][3];
    for (int c = 0; c < 3; ++c) {
        const double *u = e[(c + 1) % 3], *v = e[(c + 2) % 3];
        cr[c][0] = u[1] * v[2] - u[2] * v[1];
        cr[c][1] = u[2] * v[0] - u[0] * v[2];
        cr[c][2] = u[0] * v[1] - u[1] * v[0];
    }
    const double det = e[0][0] * cr[0][0] + e[0][1] * cr[0][1] + e[0][2] * cr[0][2];
    if (!(det > 0.0)) return false;
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) g[c + 1][r] = cr[c][r] / det;
    for (int r = 0; r < 3; ++r) g[0][r] = -(g[1][r] + g[2][r] + g[3][r]);
    *meas = det / 6.0;
    return true;
}

__host__ __device__ inline int local_edges(int dim, int E[6][2])
{
    int c = 0;
    for (int a = 0; a <= dim; ++a)
        for (int b = a + 1; b <= dim; ++b) {
            E[c][0] = a;
            E[c][1] = b;
            ++c;
        }
    return c;
}

__host__ __device__ inline bool element_matrix(int dim, int order, const double *P, double *K)
{
    double g[4][3] = {}, T;
    if (!simplex_grads(dim, P, g, &T)) return false;
    const int nv = dim + 1;
    double G[4][4];
    for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
            double s = 0.0;
            for (int r = 0; r < dim; ++r) s += g[a][r] * g[b][r];
            G[a][b] = s;
        }
    if (order == 1) {
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) K[a * nv + b] = T * G[a][b];
        return true;
    }
    const double m1 = T / (dim + 1);                           // integral l_a
    const double m2o = T / ((dim + 1.0) * (dim + 2.0));        // integral l_a l_b, a != b
    auto m2 = [m2o](int a, int b) { return a == b ? 2.0 * m2o : m2o; };
    int E[6][2];
    const int ne = local_edges(dim, E);
    const int nl = nv + ne;
    // vertex-vertex: (g_a.g_b) integral (4 l_a - 1)(4 l_b - 1)
    for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b)
            K[a * nl + b] = G[a][b] * (16.0 * m2(a, b) - 8.0 * m1 + T);
    // vertex-edge: integral (4 l_v - 1) g_v . 4 (l_a g_b + l_b g_a)
    for (int v = 0; v < nv; ++v)
        for (int e = 0; e < ne; ++e) {
            const int a = E[e][0], b = E[e][1];
            const double val = 4.0 * (G[v][b] * (4.0 * m2(v, a) - m1) + G[v][a] * (4.0 * m2(v, b) - m1));
            K[v * nl + nv + e] = val;
            K[(nv + e) * nl + v] = val;
        }
    // edge-edge: 16 integral (l_a g_b + l_b g_a).(l_c g_d + l_d g_c)
    for (int e = 0; e < ne; ++e)
        for (int f = 0; f < ne; ++f) {
            const int a = E[e][0], b = E[e][1], c = E[f][0], d = E[f][1];
            K[(nv + e) * nl + nv + f] =
                16.0 * (m2(a, c) * G[b][d] + m2(a, d) * G[b][c] + m2(b, c) * G[a][d] + m2(b, d) * G[a][c]);
        }
    return true;
}

}  // namespace femcg
