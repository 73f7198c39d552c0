/*
 * Oracle: small dense matrix exponential.  TEST INFRASTRUCTURE ONLY.
 *
 * Alg. 1 step 2 obtains phi_p(tau H_m) e_1 and phi_{p+1}(tau H_m) e_1 from
 * the exponential of an augmented matrix (remark after Alg. 1).  The cost
 * model eq. cost prices that exponential at (44/3 + 2 s) K^3 flops with
 * s = round(log2(||tau H||/5.37)), which is the flop count of a degree-13
 * Pade approximant with scaling and squaring (6 products, one LU solve, s
 * squarings).  This file is that method, written plainly:
 *
 *   s    = smallest s >= 0 with ||A||_1 / 2^s <= theta_13 = 5.371920351148152
 *   B    = A / 2^s
 *   r(B) = q(B)^-1 p(B),  p(x) = sum_j b_j x^j,  q(x) = p(-x),
 *   b_j  = (26-j)! 13! / (26! j! (13-j)!)
 *   X    = r(B)^(2^s)
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static void matmul(int K, const double *A, const double *B, double *C)
{
    for (int i = 0; i < K; i++)
        for (int j = 0; j < K; j++) {
            double acc = 0.0;
            for (int k = 0; k < K; k++) acc += A[i * K + k] * B[k * K + j];
            C[i * K + j] = acc;
        }
}

/* solve M X = R for K right-hand sides (columns of R), LU with partial pivoting */
static int lu_solve(int K, double *M, double *R)
{
    for (int c = 0; c < K; c++) {
        int piv = c;
        double best = fabs(M[c * K + c]);
        for (int r = c + 1; r < K; r++)
            if (fabs(M[r * K + c]) > best) {
                best = fabs(M[r * K + c]);
                piv = r;
            }
        if (best == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < K; k++) {
                double t = M[c * K + k]; M[c * K + k] = M[piv * K + k]; M[piv * K + k] = t;
                t = R[c * K + k]; R[c * K + k] = R[piv * K + k]; R[piv * K + k] = t;
            }
        }
        for (int r = c + 1; r < K; r++) {
            double l = M[r * K + c] / M[c * K + c];
            M[r * K + c] = l;
            for (int k = c + 1; k < K; k++) M[r * K + k] -= l * M[c * K + k];
            for (int k = 0; k < K; k++) R[r * K + k] -= l * R[c * K + k];
        }
    }
    for (int r = K - 1; r >= 0; r--)
        for (int k = 0; k < K; k++) {
            double acc = R[r * K + k];
            for (int c = r + 1; c < K; c++) acc -= M[r * K + c] * R[c * K + k];
            R[r * K + k] = acc / M[r * K + r];
        }
    return 0;
}

int orc_expm(int K, const double *A, double *X)
{
    const double theta13 = 5.371920351148152;
    size_t sz = sizeof(double) * (size_t)K * K;
    double *B = malloc(sz), *B2 = malloc(sz), *B4 = malloc(sz), *B6 = malloc(sz),
           *T = malloc(sz), *U = malloc(sz), *V = malloc(sz);

    double nrm = 0.0;
    for (int j = 0; j < K; j++) {
        double c = 0.0;
        for (int i = 0; i < K; i++) c += fabs(A[i * K + j]);
        if (c > nrm) nrm = c;
    }
    int s = 0;
    double scale = 1.0;
    while (nrm * scale > theta13) {
        s++;
        scale /= 2.0;
    }
    for (int k = 0; k < K * K; k++) B[k] = A[k] * scale;

    /* Pade numerator coefficients, b_0 = 1, b_{j+1} = b_j (13-j) / ((26-j)(j+1)) */
    double b[14];
    b[0] = 1.0;
    for (int j = 0; j < 13; j++) b[j + 1] = b[j] * (13.0 - j) / ((26.0 - j) * (j + 1.0));

    matmul(K, B, B, B2);
    matmul(K, B2, B2, B4);
    matmul(K, B4, B2, B6);
    /* odd part U = B (B6 (b13 B6 + b11 B4 + b9 B2) + b7 B6 + b5 B4 + b3 B2 + b1 I) */
    for (int k = 0; k < K * K; k++) T[k] = b[13] * B6[k] + b[11] * B4[k] + b[9] * B2[k];
    matmul(K, B6, T, U);
    for (int k = 0; k < K * K; k++) U[k] += b[7] * B6[k] + b[5] * B4[k] + b[3] * B2[k];
    for (int i = 0; i < K; i++) U[i * K + i] += b[1];
    matmul(K, B, U, T);
    memcpy(U, T, sz);
    /* even part V = B6 (b12 B6 + b10 B4 + b8 B2) + b6 B6 + b4 B4 + b2 B2 + b0 I */
    for (int k = 0; k < K * K; k++) T[k] = b[12] * B6[k] + b[10] * B4[k] + b[8] * B2[k];
    matmul(K, B6, T, V);
    for (int k = 0; k < K * K; k++) V[k] += b[6] * B6[k] + b[4] * B4[k] + b[2] * B2[k];
    for (int i = 0; i < K; i++) V[i * K + i] += b[0];
    /* (V - U) X = (V + U) */
    for (int k = 0; k < K * K; k++) {
        T[k] = V[k] - U[k];
        X[k] = V[k] + U[k];
    }
    lu_solve(K, T, X);
    for (int q = 0; q < s; q++) {
        matmul(K, X, X, T);
        memcpy(X, T, sz);
    }
    free(B); free(B2); free(B4); free(B6); free(T); free(U); free(V);
    return s;
}
