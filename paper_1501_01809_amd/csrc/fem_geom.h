// Affine simplex geometry shared by the cell kernels: the metric
// G[mn] = |det J| grad(l_m).grad(l_n) (m <= n, lexicographic) from the rows
// of adj(J), and |det J|.
#pragma once
#include <hip/hip_runtime.h>

namespace femk {

template <int D> struct Geo;

template <> struct Geo<2> {
    static constexpr int NM = 6;
    // Metric G[mn] = |det J| grad(l_m).grad(l_n) for m <= n (lexicographic);
    // returns |det J|.
    __device__ __forceinline__ static double metric(const double (&x)[3][2], double (&G)[NM])
    {
        const double c1x = x[1][0] - x[0][0], c1y = x[1][1] - x[0][1];
        const double c2x = x[2][0] - x[0][0], c2y = x[2][1] - x[0][1];
        const double det = c1x * c2y - c1y * c2x;
        // rows of adj(J): J^{-1} = adj(J) / det
        const double a[3][2] = {{-(c2y - c1y), -(c1x - c2x)}, {c2y, -c2x}, {-c1y, c1x}};
        const double adet = fabs(det), inv = 1.0 / adet;
        int t = 0;
        for (int m = 0; m < 3; ++m)
            for (int n = m; n < 3; ++n) G[t++] = (a[m][0] * a[n][0] + a[m][1] * a[n][1]) * inv;
        return adet;
    }
    __device__ __forceinline__ static double absdet(const double (&x)[3][2])
    {
        const double c1x = x[1][0] - x[0][0], c1y = x[1][1] - x[0][1];
        const double c2x = x[2][0] - x[0][0], c2y = x[2][1] - x[0][1];
        return fabs(c1x * c2y - c1y * c2x);
    }
};

template <> struct Geo<3> {
    static constexpr int NM = 10;
    __device__ __forceinline__ static double metric(const double (&x)[4][3], double (&G)[NM])
    {
        double c[3][3];
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) c[k][r] = x[k + 1][r] - x[0][r];
        double a[4][3];
        // rows of adj(J) for J = [c1 c2 c3]: c2 x c3, c3 x c1, c1 x c2
        a[1][0] = c[1][1] * c[2][2] - c[1][2] * c[2][1];
        a[1][1] = c[1][2] * c[2][0] - c[1][0] * c[2][2];
        a[1][2] = c[1][0] * c[2][1] - c[1][1] * c[2][0];
        a[2][0] = c[2][1] * c[0][2] - c[2][2] * c[0][1];
        a[2][1] = c[2][2] * c[0][0] - c[2][0] * c[0][2];
        a[2][2] = c[2][0] * c[0][1] - c[2][1] * c[0][0];
        a[3][0] = c[0][1] * c[1][2] - c[0][2] * c[1][1];
        a[3][1] = c[0][2] * c[1][0] - c[0][0] * c[1][2];
        a[3][2] = c[0][0] * c[1][1] - c[0][1] * c[1][0];
        const double det = c[0][0] * a[1][0] + c[0][1] * a[1][1] + c[0][2] * a[1][2];
        for (int r = 0; r < 3; ++r) a[0][r] = -(a[1][r] + a[2][r] + a[3][r]);
        const double adet = fabs(det), inv = 1.0 / adet;
        int t = 0;
        for (int m = 0; m < 4; ++m)
            for (int n = m; n < 4; ++n)
                G[t++] = (a[m][0] * a[n][0] + a[m][1] * a[n][1] + a[m][2] * a[n][2]) * inv;
        return adet;
    }
    __device__ __forceinline__ static double absdet(const double (&x)[4][3])
    {
        const double c1x = x[1][0] - x[0][0], c1y = x[1][1] - x[0][1], c1z = x[1][2] - x[0][2];
        const double c2x = x[2][0] - x[0][0], c2y = x[2][1] - x[0][1], c2z = x[2][2] - x[0][2];
        const double c3x = x[3][0] - x[0][0], c3y = x[3][1] - x[0][1], c3z = x[3][2] - x[0][2];
        return fabs(c1x * (c2y * c3z - c2z * c3y) - c1y * (c2x * c3z - c2z * c3x) +
                    c1z * (c2x * c3y - c2y * c3x));
    }
};

}  // namespace femk
