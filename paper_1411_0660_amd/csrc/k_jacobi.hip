// k_jacobi.hip -- eigenpairs of the small dense symmetric matrices of the
// Krylov iteration (the projected matrix of every Rayleigh-Ritz step, order
// m ~ 50 ... 600) on one gfx950 workgroup, by the cyclic two-sided Jacobi
// method (Jacobi 1846; Golub & Van Loan, Matrix Computations, section 8.5)
// with the round-robin parallel ordering (Brent & Luk 1985).
//
// A sweep is m' - 1 rounds (m' = m rounded up to even).  In round r the m'
// indices are split into m'/2 disjoint pairs by the circle method: index 0
// stays fixed and 1 ... m'-1 rotate by r, so every pair of indices meets in
// exactly one round of a sweep.  The rotations of one round commute, so they
// are applied together: one thread per pair computes its rotation from the
// 2 x 2 diagonal block, then every 2 x 2 block (k1, k2) of the matrix is
// replaced by J_k1^T A_k1k2 J_k2 by one thread, and every pair of columns of
// the accumulated vectors V by one thread per row.  Sweeps stop when a whole
// sweep found no off-diagonal entry above the threshold.
//
// The matrix and the accumulated rotations both stay in LDS when they fit
// (m <= 90), the matrix alone when it does (m <= 128: 128 KB), otherwise they
// live in their global buffers, where the workgroup's barriers order the
// accesses of its threads (one workgroup, one L1).
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace mbl {
namespace {

constexpr int JT = 1024;                // threads of the workgroup
constexpr int JLDS_MAX = 128;           // largest order kept in LDS
constexpr int JMAX = 1024;              // largest order supported
constexpr int JMAX_SWEEPS = 40;
constexpr int VB = 8;                   // V items per thread with loads in flight together

// index pair k of round r of the circle schedule over mp (even) indices
__device__ __forceinline__ void round_pair(int mp, int r, int k, int &p, int &q) {
    const int rot = mp - 1;
    int a = (k == 0) ? 0 : 1 + (k - 1 + r) % rot;
    int kb = mp - 1 - k;
    int b = 1 + (kb - 1 + r) % rot;     // kb >= 1 for every k < mp / 2
    p = min(a, b);
    q = max(a, b);
}

// Inlined at two call sites (matrix in LDS, matrix in global memory), so each
// copy addresses its matrix directly.
__device__ __forceinline__ void jacobi_rounds(int m, double *T, double *V, double *w, int *info, double tol_abs,
                              double *cs_c, double *cs_s, double *cs_t, double *cs_a, int *pp,
                              int *pq, int *nrot) {
    const int mp = m + (m & 1), nh = mp / 2;
    const int tid = threadIdx.x;
    int sweep = 0;
    for (; sweep < JMAX_SWEEPS; sweep++) {
        if (tid == 0) *nrot = 0;
        __syncthreads();
        for (int r = 0; r < mp - 1; r++) {
            // rotation of every pair of this round
            for (int k = tid; k < nh; k += JT) {
                int p, q;
                round_pair(mp, r, k, p, q);
                double c = 1.0, s = 0.0, t = 0.0, apq = 0.0;
                if (q < m) {
                    apq = T[p + (int64_t)q * m];
                    if (fabs(apq) > tol_abs) {
                        double app = T[p + (int64_t)p * m], aqq = T[q + (int64_t)q * m];
                        double theta = (aqq - app) / (2.0 * apq);
                        double at = fabs(theta);
                        t = (at > 1e150) ? 0.5 / theta
                                         : copysign(1.0, theta) / (at + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                cs_c[k] = c; cs_s[k] = s; cs_t[k] = t; cs_a[k] = apq;
                pp[k] = p; pq[k] = q;
                // rotations of this wave (s == 0 is the identity: nothing moves)
                const unsigned long long rot = __ballot(s != 0.0);
                if ((tid & 63) == 0 && rot) atomicAdd(nrot, __popcll(rot));
            }
            __syncthreads();
            // T <- J^T T J, one 2 x 2 block (and its transpose) per item; the
            // items are the pairs k1 <= k2, numbered column by column
            for (int it = tid; it < nh * (nh + 1) / 2; it += JT) {
                int k2 = (int)((sqrtf(8.0f * (float)it + 1.0f) - 1.0f) * 0.5f);
                while (k2 * (k2 + 1) / 2 > it) k2--;
                while ((k2 + 1) * (k2 + 2) / 2 <= it) k2++;
                const int k1 = it - k2 * (k2 + 1) / 2;
                const double s1 = cs_s[k1], s2 = cs_s[k2];
                if (s1 == 0.0 && s2 == 0.0) continue;
                const int p1 = pp[k1], q1 = pq[k1], p2 = pp[k2], q2 = pq[k2];
                if (k1 == k2) {                  // the rotated pair itself: diagonalised
                    const double t = cs_t[k1], apq = cs_a[k1];
                    T[p1 + (int64_t)p1 * m] -= t * apq;
                    T[q1 + (int64_t)q1 * m] += t * apq;
                    T[p1 + (int64_t)q1 * m] = 0.0;
                    T[q1 + (int64_t)p1 * m] = 0.0;
                    continue;
                }
                const double c1 = cs_c[k1], c2 = cs_c[k2];
                const bool vq1 = q1 < m, vq2 = q2 < m;
                double x = T[p1 + (int64_t)p2 * m];
                double y = vq2 ? T[p1 + (int64_t)q2 * m] : 0.0;
                double z = vq1 ? T[q1 + (int64_t)p2 * m] : 0.0;
                double u = (vq1 && vq2) ? T[q1 + (int64_t)q2 * m] : 0.0;
                // columns (p2, q2)
                double x1 = c2 * x - s2 * y, y1 = s2 * x + c2 * y;
                double z1 = c2 * z - s2 * u, u1 = s2 * z + c2 * u;
                // rows (p1, q1)
                double x2 = c1 * x1 - s1 * z1, z2 = s1 * x1 + c1 * z1;
                double y2 = c1 * y1 - s1 * u1, u2 = s1 * y1 + c1 * u1;
                T[p1 + (int64_t)p2 * m] = x2;
                T[p2 + (int64_t)p1 * m] = x2;
                if (vq2) { T[p1 + (int64_t)q2 * m] = y2; T[q2 + (int64_t)p1 * m] = y2; }
                if (vq1) { T[q1 + (int64_t)p2 * m] = z2; T[p2 + (int64_t)q1 * m] = z2; }
                if (vq1 && vq2) { T[q1 + (int64_t)q2 * m] = u2; T[q2 + (int64_t)q1 * m] = u2; }
            }
            // V <- V J, one row of one column pair per item; items are taken
            // VB at a time with all their loads issued before any store, since
            // V lives in global memory (L2) and each load is a round trip
            for (int base = 0; base < m * nh; base += VB * JT) {
                double va[VB], vb[VB];
#pragma unroll
                for (int u = 0; u < VB; u++) {
                    const int it = base + u * JT + tid;
                    va[u] = vb[u] = 0.0;
                    if (it < m * nh) {
                        const int i = it % m, k = it / m;
                        if (cs_s[k] != 0.0) {
                            va[u] = V[(int64_t)pp[k] * m + i];
                            vb[u] = V[(int64_t)pq[k] * m + i];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < VB; u++) {
                    const int it = base + u * JT + tid;
                    if (it >= m * nh) continue;
                    const int i = it % m, k = it / m;
                    const double s = cs_s[k];
                    if (s == 0.0) continue;
                    const double c = cs_c[k];
                    V[(int64_t)pp[k] * m + i] = c * va[u] - s * vb[u];
                    V[(int64_t)pq[k] * m + i] = s * va[u] + c * vb[u];
                }
            }
            __syncthreads();
        }
        if (*nrot == 0) break;
        __syncthreads();
    }
    for (int i = tid; i < m; i += JT) w[i] = T[i + (int64_t)i * m];
    if (tid == 0) *info = (sweep < JMAX_SWEEPS) ? sweep : -1;
}

// A (m x m, column-major, symmetric; overwritten), V (m x m) <- eigenvectors,
// w[m] <- eigenvalues (unsorted, w[j] belongs to column j of V),
// info <- sweeps used, or -1 if the sweep limit was reached.
// Matrix blockIdx.x of a batch: operands at strides m^2 (A, V), m (w), 1
// (info); its threshold tol_abs[blockIdx.x].
__global__ __launch_bounds__(JT) void k_jacobi_eig(int m, double *A, double *V, double *w,
                                                   int *info, const double *tol) {
    __shared__ double Tl[JLDS_MAX * JLDS_MAX];
    __shared__ double cs_c[JMAX / 2], cs_s[JMAX / 2], cs_t[JMAX / 2], cs_a[JMAX / 2];
    __shared__ int pp[JMAX / 2], pq[JMAX / 2], nrot;
    const int64_t mm = (int64_t)m * m;
    A += blockIdx.x * mm;
    V += blockIdx.x * mm;
    w += (int64_t)blockIdx.x * m;
    info += blockIdx.x;
    const double tol_abs = tol[blockIdx.x];
    if (2 * mm <= JLDS_MAX * JLDS_MAX) {
        // both the matrix and the accumulated rotations in LDS (m <= 90)
        double *Vl = Tl + mm;
        for (int it = threadIdx.x; it < m * m; it += JT) {
            Tl[it] = A[it];
            Vl[it] = ((it % m) == (it / m)) ? 1.0 : 0.0;
        }
        __syncthreads();
        jacobi_rounds(m, Tl, Vl, w, info, tol_abs, cs_c, cs_s, cs_t, cs_a, pp, pq, &nrot);
        __syncthreads();
        for (int it = threadIdx.x; it < m * m; it += JT) V[it] = Vl[it];
        return;
    }
    for (int it = threadIdx.x; it < m * m; it += JT)
        V[it] = ((it % m) == (it / m)) ? 1.0 : 0.0;
    if (m <= JLDS_MAX) {
        for (int it = threadIdx.x; it < m * m; it += JT) Tl[it] = A[it];
        __syncthreads();
        jacobi_rounds(m, Tl, V, w, info, tol_abs, cs_c, cs_s, cs_t, cs_a, pp, pq, &nrot);
    } else {
        __syncthreads();
        jacobi_rounds(m, A, V, w, info, tol_abs, cs_c, cs_s, cs_t, cs_a, pp, pq, &nrot);
    }
}

}  // namespace

void launch_jacobi_eig_batch(int count, int m, double *A, double *V, double *w, int *info,
                             const double *tol_abs, hipStream_t s) {
    MBL_REQUIRE(m >= 1 && m <= JMAX, MBL_EINVAL, "Jacobi eigensolver: order out of range");
    if (count == 0) return;
    hipLaunchKernelGGL(k_jacobi_eig, dim3(count), dim3(JT), 0, s, m, A, V, w, info, tol_abs);
    MBL_CHECK_LAUNCH();
}

}  // namespace mbl
