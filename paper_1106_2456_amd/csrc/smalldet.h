// Small determinants of table entries and their bordered derivative terms.
//
// For an excitation of order k with holes h_j and particles p_j the ratio of
// the excited determinant to the reference is det S, S[j][l] = T[h_j][p_l]
// (Sec. III, the r x r read-off).  The derivative with respect to electron i
// of the excited determinant, relative to the reference at R', is the
// bordered determinant
//     rho^a det S + g^a[p]^T adj(S) c'[h]
// (Sec. IV-A table of the row-replaced reference written without inverting
// it; equal to Sec. IV-C's lemma at rank one).  So per excitation we need
// det S and y = adj(S) c'[h]; y_j = det(S with column j replaced by c'[h])
// (Cramer), which stays finite when S is singular.
//
// The routines take S by columns: col[j][r] = S[r][j] = T[h_r][p_j].  Orders
// 1..4 are written out with shared 2 x 2 minors (Laplace expansion); orders
// 5..8 use Gaussian elimination with partial pivoting on k + 1 matrices.
// Compiled for the device (HIP) and, in a host-only test build, for the CPU.
#pragma once

#if defined(__HIPCC__)
#define MDE_HD __host__ __device__ __forceinline__
#else
#define MDE_HD inline
#endif

namespace mde {

// det of a k x k matrix given by columns; generic path (k <= 8)
template <typename F>
MDE_HD F det_generic(int k, F a[8][8]) {
    // a[c][r]: column c, row r; destroyed
    F det = F(1);
    for (int c = 0; c < k; ++c) {
        int p = c;
        F best = a[c][c] < F(0) ? -a[c][c] : a[c][c];
        for (int r = c + 1; r < k; ++r) {
            F v = a[c][r] < F(0) ? -a[c][r] : a[c][r];
            if (v > best) { best = v; p = r; }
        }
        if (best == F(0)) return F(0);
        if (p != c) {
            for (int cc = 0; cc < k; ++cc) { F t = a[cc][c]; a[cc][c] = a[cc][p]; a[cc][p] = t; }
            det = -det;
        }
        F piv = a[c][c];
        det *= piv;
        for (int r = c + 1; r < k; ++r) {
            F f = a[c][r] / piv;
            for (int cc = c + 1; cc < k; ++cc) a[cc][r] -= f * a[cc][c];
        }
    }
    return det;
}

// Order K: given columns col[j][r] and c[r], returns det S and y[j].
template <int K, typename F>
struct SmallDet;

template <typename F>
struct SmallDet<1, F> {
    MDE_HD static F run(const F col[1][1], const F c[1], F y[1]) {
        y[0] = c[0];
        return col[0][0];
    }
};

template <typename F>
struct SmallDet<2, F> {
    MDE_HD static F run(const F col[2][2], const F c[2], F y[2]) {
        // det(a, b) with a, b columns: a0 b1 - b0 a1
        F det = col[0][0] * col[1][1] - col[1][0] * col[0][1];
        y[0] = c[0] * col[1][1] - col[1][0] * c[1];
        y[1] = col[0][0] * c[1] - c[0] * col[0][1];
        return det;
    }
};

template <typename F>
struct SmallDet<3, F> {
    MDE_HD static F run(const F col[3][3], const F c[3], F y[3]) {
        // minors of rows 1,2: m(x, z) = x1 z2 - z1 x2, expansion along row 0
        const F *C0 = col[0], *C1 = col[1], *C2 = col[2];
        F m12 = C1[1] * C2[2] - C2[1] * C1[2];
        F m02 = C0[1] * C2[2] - C2[1] * C0[2];
        F m01 = C0[1] * C1[2] - C1[1] * C0[2];
        F mc0 = c[1] * C0[2] - C0[1] * c[2];   // m(c, C0)
        F mc1 = c[1] * C1[2] - C1[1] * c[2];
        F mc2 = c[1] * C2[2] - C2[1] * c[2];
        F det = C0[0] * m12 - C1[0] * m02 + C2[0] * m01;
        y[0] = c[0] * m12 - C1[0] * mc2 + C2[0] * mc1;     // det(c, C1, C2)
        y[1] = C0[0] * mc2 - c[0] * m02 - C2[0] * mc0;     // det(C0, c, C2)
        y[2] = -C0[0] * mc1 + C1[0] * mc0 + c[0] * m01;    // det(C0, C1, c)
        return det;
    }
};

template <typename F>
struct SmallDet<4, F> {
    MDE_HD static F run(const F col[4][4], const F c[4], F y[4]) {
        // Laplace expansion along rows (0,1) x rows (2,3):
        // det = t01 b23 - t02 b13 + t03 b12 + t12 b03 - t13 b02 + t23 b01
        // t(x,z) = x0 z1 - z0 x1 (top rows), b(x,z) = x2 z3 - z2 x3 (bottom)
        const F *C0 = col[0], *C1 = col[1], *C2 = col[2], *C3 = col[3];
        F t01 = C0[0] * C1[1] - C1[0] * C0[1], b01 = C0[2] * C1[3] - C1[2] * C0[3];
        F t02 = C0[0] * C2[1] - C2[0] * C0[1], b02 = C0[2] * C2[3] - C2[2] * C0[3];
        F t03 = C0[0] * C3[1] - C3[0] * C0[1], b03 = C0[2] * C3[3] - C3[2] * C0[3];
        F t12 = C1[0] * C2[1] - C2[0] * C1[1], b12 = C1[2] * C2[3] - C2[2] * C1[3];
        F t13 = C1[0] * C3[1] - C3[0] * C1[1], b13 = C1[2] * C3[3] - C3[2] * C1[3];
        F t23 = C2[0] * C3[1] - C3[0] * C2[1], b23 = C2[2] * C3[3] - C3[2] * C2[3];
        // minors with the replacement column c first: t(c, Cj), b(c, Cj)
        F tc0 = c[0] * C0[1] - C0[0] * c[1], bc0 = c[2] * C0[3] - C0[2] * c[3];
        F tc1 = c[0] * C1[1] - C1[0] * c[1], bc1 = c[2] * C1[3] - C1[2] * c[3];
        F tc2 = c[0] * C2[1] - C2[0] * c[1], bc2 = c[2] * C2[3] - C2[2] * c[3];
        F tc3 = c[0] * C3[1] - C3[0] * c[1], bc3 = c[2] * C3[3] - C3[2] * c[3];
        F det = t01 * b23 - t02 * b13 + t03 * b12 + t12 * b03 - t13 * b02 + t23 * b01;
        // column j -> c: every pair holding j uses t/b with c in j's place,
        // t(Ci, c) = -t(c, Ci)
        y[0] = tc1 * b23 - tc2 * b13 + tc3 * b12 + t12 * bc3 - t13 * bc2 + t23 * bc1;
        y[1] = -tc0 * b23 - t02 * bc3 + t03 * bc2 + tc2 * b03 - tc3 * b02 - t23 * bc0;
        y[2] = t01 * bc3 + tc0 * b13 - t03 * bc1 - tc1 * b03 + t13 * bc0 + tc3 * b01;
        y[3] = -t01 * bc2 + t02 * bc1 - tc0 * b12 - t12 * bc0 + tc1 * b02 - tc2 * b01;
        return det;
    }
};

// Generic order k (5..8): det S and y_j = det(S with column j -> c).
template <typename F>
MDE_HD F small_det_generic(int k, const F col[8][8], const F c[8], F y[8]) {
    F a[8][8];
    for (int j = 0; j < k; ++j)
        for (int r = 0; r < k; ++r) a[j][r] = col[j][r];
    F det = det_generic<F>(k, a);
    for (int jj = 0; jj < k; ++jj) {
        for (int j = 0; j < k; ++j)
            for (int r = 0; r < k; ++r) a[j][r] = (j == jj) ? c[r] : col[j][r];
        y[jj] = det_generic<F>(k, a);
    }
    return det;
}

// Run form.  With the first K-1 columns P_0..P_{K-2} of S fixed, det S is
// linear in the last column b: det [P_0 .. P_{K-2}, b] = u . b, u the
// cofactors of the last column (1; a 2-d rotation; the cross product; the
// 4-d cross product from the 2 x 2 minors of the first two columns).
template <typename F>
MDE_HD void cross4(const F x[4], const F y[4], const F z[4], F w[4]) {
    const F m01 = x[0] * y[1] - x[1] * y[0], m02 = x[0] * y[2] - x[2] * y[0];
    const F m03 = x[0] * y[3] - x[3] * y[0], m12 = x[1] * y[2] - x[2] * y[1];
    const F m13 = x[1] * y[3] - x[3] * y[1], m23 = x[2] * y[3] - x[3] * y[2];
    w[0] = -m12 * z[3] + m13 * z[2] - m23 * z[1];
    w[1] = m02 * z[3] - m03 * z[2] + m23 * z[0];
    w[2] = -m01 * z[3] + m03 * z[1] - m13 * z[0];
    w[3] = m01 * z[2] - m02 * z[1] + m12 * z[0];
}

template <int K, typename F>
MDE_HD void last_cofactors(const F P[(K > 1 ? K - 1 : 1)][K], F u[K]) {
    if constexpr (K == 1) {
        u[0] = F(1);
    } else if constexpr (K == 2) {
        u[0] = -P[0][1];
        u[1] = P[0][0];
    } else if constexpr (K == 3) {
        u[0] = P[0][1] * P[1][2] - P[0][2] * P[1][1];
        u[1] = P[0][2] * P[1][0] - P[0][0] * P[1][2];
        u[2] = P[0][0] * P[1][1] - P[0][1] * P[1][0];
    } else {
        static_assert(K == 4, "run form is written for orders 1..4");
        cross4<F>(P[0], P[1], P[2], u);
    }
}

// y_j = det(S with column j replaced by c) for j < K-1 is v_j . b with v_j
// the last-column cofactors of the prefix whose column j is c; y_{K-1} = u . c.
template <int K, typename F>
MDE_HD void prefix_cofactors(const F P[(K > 1 ? K - 1 : 1)][K], const F c[K], F u[K],
                             F v[(K > 1 ? K - 1 : 1)][K], F &ylast) {
    constexpr int KP = K - 1, KQ = K > 1 ? K - 1 : 1;
    last_cofactors<K, F>(P, u);
    for (int j = 0; j < KP; ++j) {
        F Q[KQ][K];
        for (int i = 0; i < KP; ++i)
            for (int r = 0; r < K; ++r) Q[i][r] = (i == j) ? c[r] : P[i][r];
        last_cofactors<K, F>(Q, v[j]);
    }
    F s = F(0);
    for (int r = 0; r < K; ++r) s += u[r] * c[r];
    ylast = s;
}

}  // namespace mde
