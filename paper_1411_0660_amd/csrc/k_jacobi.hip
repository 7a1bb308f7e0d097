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
// Orders up to 128 (the projected matrices of nev up to about 55) run in
// k_jacobi_lds: the matrix in LDS with an odd leading dimension (few bank
// conflicts along rows as along columns), the accumulated rotations in LDS
// too up to order 90, work found through tables, every thread's loads of a
// round issued before its stores.
// Larger orders run in k_jacobi_eig, with the matrix and the rotations in
// their global buffers (it also keeps the matrix in LDS when asked to run an
// order up to 128).  Both kernels apply the same rotations with the same
// arithmetic, element by element, so they give the same results bit for bit.
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

// Every fused multiply-add below is written out; no other is formed, so the
// rounding of each update is fixed by the source and the two kernels, which
// apply the same rotations, agree bit for bit.
#pragma clang fp contract(off)

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

// J_1^T [x y; z u] J_2 for the 2 x 2 block of rows (p1, q1) and columns
// (p2, q2): the column pair rotated by (c2, s2), then the row pair by (c1, s1)
__device__ __forceinline__ void rotate_block(double c1, double s1, double c2, double s2, double x,
                                             double y, double z, double u, double &x2, double &y2,
                                             double &z2, double &u2) {
    const double x1 = fma(c2, x, -(s2 * y)), y1 = fma(s2, x, c2 * y);
    const double z1 = fma(c2, z, -(s2 * u)), u1 = fma(s2, z, c2 * u);
    x2 = fma(c1, x1, -(s1 * z1));
    z2 = fma(s1, x1, c1 * z1);
    y2 = fma(c1, y1, -(s1 * u1));
    u2 = fma(s1, y1, c1 * u1);
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
                                         : copysign(1.0, theta) / (at + sqrt(fma(theta, theta, 1.0)));
                        c = 1.0 / sqrt(fma(t, t, 1.0));
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
                    T[p1 + (int64_t)p1 * m] = fma(-t, apq, T[p1 + (int64_t)p1 * m]);
                    T[q1 + (int64_t)q1 * m] = fma(t, apq, T[q1 + (int64_t)q1 * m]);
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
                double x2, y2, z2, u2;
                rotate_block(c1, s1, c2, s2, x, y, z, u, x2, y2, z2, u2);
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
                    V[(int64_t)pp[k] * m + i] = fma(c, va[u], -(s * vb[u]));
                    V[(int64_t)pq[k] * m + i] = fma(s, va[u], c * vb[u]);
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

constexpr int JL_T = 1024;              // threads of the LDS kernel
constexpr int JL_VMAX = 90;             // largest order with the rotations in LDS too
constexpr int JL_MAX = 128;             // largest order of the matrix in LDS

// Pair k (< mp / 2) of round r of the circle schedule over mp (even) indices.
__device__ __forceinline__ void circle_pair(int mp, int r, int k, int &p, int &q) {
    const int rot = mp - 1;
    int a = 0;
    if (k > 0) {
        a = k - 1 + r;
        if (a >= rot) a -= rot;
        a += 1;
    }
    int b = mp - 2 - k + r;
    if (b >= rot) b -= rot;
    b += 1;
    p = min(a, b);
    q = max(a, b);
}

// Same contract and results as k_jacobi_eig, for m <= MAXM.  The matrix is
// kept with an odd leading dimension ld, so that a row of it, like a column,
// spreads over the LDS banks: the 2 x 2 block update reads blocks along
// columns and stores their transposes along rows.  The accumulated rotations
// are in LDS too (VL) when both fit, else in their global buffer (the
// workgroup's barriers order its threads' accesses: one workgroup, one L1).
// The blocks (and the V items) are numbered once, in tables, so a thread
// finds its work without division; each thread issues all loads of its items
// before any store.
template <int MAXM, bool VL>
__global__ __launch_bounds__(JL_T) void k_jacobi_lds(int m, const double *A, double *V, double *w,
                                                     int *info, const double *tol) {
    constexpr int NH = MAXM / 2;                              // pairs of a round
    constexpr int ITEMS = NH * (NH + 1) / 2;
    constexpr int IT = (ITEMS + JL_T - 1) / JL_T;             // 2 x 2 blocks per thread
    constexpr int VI = (MAXM * NH + JL_T - 1) / JL_T;         // V items per thread
    static_assert(NH <= 64, "the rotations of a round are computed by one wave");
    static_assert(NH < 256, "item table packs two pair indices in 8 bits each");
    __shared__ double T[MAXM * (MAXM + 1)], Vs[VL ? MAXM * MAXM : 1];
    __shared__ double2 cs[NH], ta[NH];             // (c, s) and (t, a_pq) of each pair
    __shared__ int pp[NH], pq[NH];
    __shared__ uint16_t item[ITEMS];               // block k1 | k2 << 8, k1 <= k2
    __shared__ int moved;
    const int64_t mm = (int64_t)m * m;
    A += blockIdx.x * mm;
    V += blockIdx.x * mm;
    w += (int64_t)blockIdx.x * m;
    info += blockIdx.x;
    const double tol_abs = tol[blockIdx.x];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int mp = m + (m & 1), nh = mp / 2, rot = mp - 1, ld = m | 1;
    const int nitems = nh * (nh + 1) / 2, nvi = m * nh;
    double *Vl = VL ? Vs : V;
    for (int it = tid; it < m * m; it += JL_T) {
        const int i = it % m, j = it / m;
        T[i + j * ld] = A[it];
        Vl[it] = (i == j) ? 1.0 : 0.0;
    }
    for (int it = tid; it < nitems; it += JL_T) {
        int k2 = (int)((sqrtf(8.0f * (float)it + 1.0f) - 1.0f) * 0.5f);
        while (k2 * (k2 + 1) / 2 > it) k2--;
        while ((k2 + 1) * (k2 + 2) / 2 <= it) k2++;
        item[it] = (uint16_t)((it - k2 * (k2 + 1) / 2) | (k2 << 8));
    }
    // V items of this thread: row vi_i[j] of pair vi_k[j] (-1: none)
    int vi_i[VI], vi_k[VI];
#pragma unroll
    for (int j = 0; j < VI; j++) {
        const int it = tid + j * JL_T;
        vi_i[j] = it < nvi ? it % m : 0;
        vi_k[j] = it < nvi ? it / m : -1;
    }
    int sweep = 0;
    for (; sweep < JMAX_SWEEPS; sweep++) {
        if (tid == 0) moved = 0;
        __syncthreads();
        for (int r = 0; r < rot; r++) {
            if (wv == 0) {
                double c = 1.0, s = 0.0, t = 0.0, apq = 0.0;
                if (lane < nh) {
                    int p, q;
                    circle_pair(mp, r, lane, p, q);
                    if (q < m) {
                        apq = T[p + q * ld];
                        if (fabs(apq) > tol_abs) {
                            double app = T[p + p * ld], aqq = T[q + q * ld];
                            double theta = (aqq - app) / (2.0 * apq);
                            double at = fabs(theta);
                            t = (at > 1e150) ? 0.5 / theta
                                             : copysign(1.0, theta) /
                                                   (at + sqrt(fma(theta, theta, 1.0)));
                            c = 1.0 / sqrt(fma(t, t, 1.0));
                            s = t * c;
                        }
                    }
                    cs[lane] = make_double2(c, s);
                    ta[lane] = make_double2(t, apq);
                    pp[lane] = p;
                    pq[lane] = q;
                }
                if (__ballot(s != 0.0) && lane == 0) moved = 1;
            }
            __syncthreads();
            // T <- J^T T J by 2 x 2 blocks: all loads first (the blocks of a
            // round are disjoint), then the stores
            {
                double x[IT], y[IT], z[IT], u[IT];
                int kk[IT];
#pragma unroll
                for (int j = 0; j < IT; j++) {
                    const int it = tid + j * JL_T;
                    kk[j] = -1;
                    if (it >= nitems) continue;
                    const int k1 = item[it] & 255, k2 = item[it] >> 8;
                    if (cs[k1].y == 0.0 && cs[k2].y == 0.0) continue;
                    kk[j] = item[it];
                    if (k1 == k2) continue;
                    const int p1 = pp[k1], q1 = pq[k1], p2 = pp[k2], q2 = pq[k2];
                    const bool vq1 = q1 < m, vq2 = q2 < m;
                    x[j] = T[p1 + p2 * ld];
                    y[j] = vq2 ? T[p1 + q2 * ld] : 0.0;
                    z[j] = vq1 ? T[q1 + p2 * ld] : 0.0;
                    u[j] = (vq1 && vq2) ? T[q1 + q2 * ld] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < IT; j++) {
                    if (kk[j] < 0) continue;
                    const int k1 = kk[j] & 255, k2 = kk[j] >> 8;
                    const int p1 = pp[k1], q1 = pq[k1];
                    if (k1 == k2) {              // the rotated pair itself: diagonalised
                        const double2 tq = ta[k1];
                        T[p1 + p1 * ld] = fma(-tq.x, tq.y, T[p1 + p1 * ld]);
                        T[q1 + q1 * ld] = fma(tq.x, tq.y, T[q1 + q1 * ld]);
                        T[p1 + q1 * ld] = 0.0;
                        T[q1 + p1 * ld] = 0.0;
                        continue;
                    }
                    const int p2 = pp[k2], q2 = pq[k2];
                    const bool vq1 = q1 < m, vq2 = q2 < m;
                    const double2 r1 = cs[k1], r2 = cs[k2];
                    double x2, y2, z2, u2;
                    rotate_block(r1.x, r1.y, r2.x, r2.y, x[j], y[j], z[j], u[j], x2, y2, z2, u2);
                    T[p1 + p2 * ld] = x2;
                    T[p2 + p1 * ld] = x2;
                    if (vq2) { T[p1 + q2 * ld] = y2; T[q2 + p1 * ld] = y2; }
                    if (vq1) { T[q1 + p2 * ld] = z2; T[p2 + q1 * ld] = z2; }
                    if (vq1 && vq2) { T[q1 + q2 * ld] = u2; T[q2 + q1 * ld] = u2; }
                }
            }
            // V <- V J, one row of one column pair per item
            {
                double va[VI], vb[VI];
#pragma unroll
                for (int j = 0; j < VI; j++) {
                    va[j] = vb[j] = 0.0;
                    const int k = vi_k[j];
                    if (k >= 0 && cs[k].y != 0.0) {
                        va[j] = Vl[pp[k] * m + vi_i[j]];
                        vb[j] = Vl[pq[k] * m + vi_i[j]];
                    }
                }
#pragma unroll
                for (int j = 0; j < VI; j++) {
                    const int k = vi_k[j];
                    if (k < 0) continue;
                    const double2 r2 = cs[k];
                    if (r2.y == 0.0) continue;
                    Vl[pp[k] * m + vi_i[j]] = fma(r2.x, va[j], -(r2.y * vb[j]));
                    Vl[pq[k] * m + vi_i[j]] = fma(r2.y, va[j], r2.x * vb[j]);
                }
            }
            __syncthreads();
        }
        if (moved == 0) break;
        __syncthreads();
    }
    for (int i = tid; i < m; i += JL_T) w[i] = T[i + i * ld];
    if (VL)
        for (int it = tid; it < m * m; it += JL_T) V[it] = Vl[it];
    if (tid == 0) *info = (sweep < JMAX_SWEEPS) ? sweep : -1;
}

}  // namespace

void launch_jacobi_eig_batch(int count, int m, double *A, double *V, double *w, int *info,
                             const double *tol_abs, hipStream_t s, bool general) {
    MBL_REQUIRE(m >= 1 && m <= JMAX, MBL_EINVAL, "Jacobi eigensolver: order out of range");
    if (count == 0) return;
    if (m <= JL_VMAX && !general)
        hipLaunchKernelGGL((k_jacobi_lds<JL_VMAX, true>), dim3(count), dim3(JL_T), 0, s, m, A, V, w,
                           info, tol_abs);
    else if (m <= JL_MAX && !general)
        hipLaunchKernelGGL((k_jacobi_lds<JL_MAX, false>), dim3(count), dim3(JL_T), 0, s, m, A, V, w,
                           info, tol_abs);
    else
        hipLaunchKernelGGL(k_jacobi_eig, dim3(count), dim3(JT), 0, s, m, A, V, w, info, tol_abs);
    MBL_CHECK_LAUNCH();
}

}  // namespace mbl
