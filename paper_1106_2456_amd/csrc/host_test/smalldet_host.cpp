// Host build of the small-determinant routines for CPU unit tests.
#include "../smalldet.h"

extern "C" double mde_host_small_det(int k, const double *S, const double *c, double *y) {
    // S row-major k x k: S[r][j]
    double col[8][8], cc[8], yy[8];
    for (int j = 0; j < k; ++j)
        for (int r = 0; r < k; ++r) col[j][r] = S[r * k + j];
    for (int r = 0; r < k; ++r) cc[r] = c[r];
    double det;
    switch (k) {
        case 1: { double C1[1][1] = {{col[0][0]}}; det = mde::SmallDet<1, double>::run(C1, cc, yy); break; }
        case 2: { double C2[2][2]; for (int j = 0; j < 2; ++j) for (int r = 0; r < 2; ++r) C2[j][r] = col[j][r];
                  det = mde::SmallDet<2, double>::run(C2, cc, yy); break; }
        case 3: { double C3[3][3]; for (int j = 0; j < 3; ++j) for (int r = 0; r < 3; ++r) C3[j][r] = col[j][r];
                  det = mde::SmallDet<3, double>::run(C3, cc, yy); break; }
        case 4: { double C4[4][4]; for (int j = 0; j < 4; ++j) for (int r = 0; r < 4; ++r) C4[j][r] = col[j][r];
                  det = mde::SmallDet<4, double>::run(C4, cc, yy); break; }
        default: det = mde::small_det_generic<double>(k, col, cc, yy); break;
    }
    for (int j = 0; j < k; ++j) y[j] = yy[j];
    return det;
}

extern "C" double mde_host_small_det_generic(int k, const double *S, const double *c, double *y) {
    double col[8][8], cc[8], yy[8];
    for (int j = 0; j < k; ++j)
        for (int r = 0; r < k; ++r) col[j][r] = S[r * k + j];
    for (int r = 0; r < k; ++r) cc[r] = c[r];
    double det = mde::small_det_generic<double>(k, col, cc, yy);
    for (int j = 0; j < k; ++j) y[j] = yy[j];
    return det;
}

// Run form: det S and y from the prefix cofactors (first k-1 columns of S)
// applied to the last column; S row-major k x k, k = 1..4.
template <int K>
static double run_form(const double *S, const double *c, double *y) {
    constexpr int KQ = K > 1 ? K - 1 : 1;
    double P[KQ][K], b[K], cc[K], u[K], v[KQ][K], ylast;
    for (int j = 0; j < K - 1; ++j)
        for (int r = 0; r < K; ++r) P[j][r] = S[r * K + j];
    for (int r = 0; r < K; ++r) {
        b[r] = S[r * K + K - 1];
        cc[r] = c[r];
    }
    mde::prefix_cofactors<K, double>(P, cc, u, v, ylast);
    double det = 0.0;
    for (int r = 0; r < K; ++r) det += u[r] * b[r];
    for (int j = 0; j < K - 1; ++j) {
        double s = 0.0;
        for (int r = 0; r < K; ++r) s += v[j][r] * b[r];
        y[j] = s;
    }
    y[K - 1] = ylast;
    return det;
}

extern "C" double mde_host_run_form(int k, const double *S, const double *c, double *y) {
    switch (k) {
        case 1: return run_form<1>(S, c, y);
        case 2: return run_form<2>(S, c, y);
        case 3: return run_form<3>(S, c, y);
        case 4: return run_form<4>(S, c, y);
        default: return 0.0;
    }
}
