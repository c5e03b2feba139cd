// Recompression of the core of a low-rank product: a batched, truncated
// singular value decomposition of small matrices, one workgroup per matrix.
//
// The product of two low-rank blocks A = A_U A_X A_V^T and B = B_U B_X B_V^T
// is A_U G B_V^T with the rank-sized core G = A_X (A_V^T B_U) B_X of Alg. 1.
// With orthonormal outer bases (the usual low-rank format) recompressing the
// product to rank k only needs the SVD of G: G = X S Y^T, truncated to the k
// largest singular values; the new bases are A_U X_k and B_V Y_k.
//
// The SVD is one-sided Jacobi (Hestenes): the columns a_p of G (m x n, both
// at most 64) are orthogonalised pairwise by plane rotations applied to G and
// to V (initially the identity), until every pair is orthogonal to working
// precision; then sigma_p = |a_p|, the left vectors are a_p / sigma_p and the
// right vectors the columns of V.  A core with fewer rows than columns is
// processed as its transpose (so exactly min(m, n) singular values come out,
// and the vectors swap roles).  Pairs follow a round-robin tournament
// (N = n rounded up to even: N - 1 steps of N / 2 disjoint pairs per sweep),
// 8 lanes per pair.  For a pair with alpha = |a_p|^2, beta = |a_q|^2,
// gamma = a_p . a_q the rotation zeta = (beta - alpha) / (2 gamma),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t,
// a_p <- c a_p - s a_q, a_q <- s a_p + c a_q makes the pair orthogonal.
#include "lrbg_tiles.h"

namespace lrbg {

constexpr int kSvdMax = 64;    // m, n <= 64
constexpr int kSvdSweeps = 40;

// One core per workgroup of 4 NMAX threads (NMAX / 2 pairs x 8 lanes), G and
// V in LDS sized for NMAX x NMAX: small cores run many workgroups per CU,
// which is what hides the latency of each rotation step.
template <int NMAX>
__global__ void __launch_bounds__(4 * NMAX)
lrbg_core_svd_kernel(const SvdDesc *__restrict__ descs, int count)
{
    constexpr int LD = NMAX + 1, NT = 4 * NMAX;
    __shared__ double A[NMAX * LD];    // column p at A + p * LD
    __shared__ double V[NMAX * LD];
    __shared__ double sig[NMAX];
    __shared__ int32_t perm[NMAX];
    __shared__ int32_t s_k;
    const int t = blockIdx.x;
    if (t >= count) return;
    const SvdDesc d = descs[t];
    const bool tr = d.m < d.n;                     // work on G^T
    const int m = tr ? d.n : d.m, n = tr ? d.m : d.n, tid = threadIdx.x;

    for (int e = tid; e < NMAX * NMAX; e += NT) {
        const int i = e % NMAX, p = e / NMAX;
        double v = 0.0;
        if (i < m && p < n) v = tr ? d.g[p + (size_t)i * d.ldg] : d.g[i + (size_t)p * d.ldg];
        A[p * LD + i] = v;
        V[p * LD + i] = (i == p) ? 1.0 : 0.0;
    }
    __syncthreads();

    const int N = (n + 1) & ~1;
    const int pairs = N / 2, pr = tid >> 3, l8 = tid & 7;
    for (int sweep = 0; sweep < kSvdSweeps && N >= 2; ++sweep) {
        int rotated = 0;
        for (int step = 0; step < N - 1; ++step) {
            if (pr < pairs) {
                // circle method: position 0 fixed, positions 1..N-1 rotate
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (N - 1); };
                int p = player(pr), q = player(N - 1 - pr);
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                if (q < n) {
                    double *ap = A + p * LD, *aq = A + q * LD;
                    double al = 0.0, be = 0.0, ga = 0.0;
                    for (int i = l8; i < m; i += 8) {
                        const double x = ap[i], y = aq[i];
                        al += x * x;
                        be += y * y;
                        ga += x * y;
                    }
#pragma unroll
                    for (int o = 4; o >= 1; o >>= 1) {
                        al += __shfl_xor(al, o, 8);
                        be += __shfl_xor(be, o, 8);
                        ga += __shfl_xor(ga, o, 8);
                    }
                    if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                        for (int i = l8; i < m; i += 8) {
                            const double x = ap[i], y = aq[i];
                            ap[i] = c * x - s * y;
                            aq[i] = s * x + c * y;
                        }
                        double *vp = V + p * LD, *vq = V + q * LD;
                        for (int i = l8; i < n; i += 8) {
                            const double x = vp[i], y = vq[i];
                            vp[i] = c * x - s * y;
                            vq[i] = s * x + c * y;
                        }
                        rotated = 1;
                    }
                }
            }
            __syncthreads();
        }
        if (!__syncthreads_or(rotated)) break;
    }

    // singular values, descending order (ties by index), truncation rank
    if (tid < n) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += A[tid * LD + i] * A[tid * LD + i];
        sig[tid] = sqrt(s2);
    }
    __syncthreads();
    if (tid < n) {
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += (sig[j] > sig[tid]) || (sig[j] == sig[tid] && j < tid);
        perm[rank] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        const double smax = n > 0 ? sig[perm[0]] : 0.0;
        int k = 0;
        while (k < n && k < d.kmax && smax > 0.0 && sig[perm[k]] > d.tol * smax) ++k;
        s_k = k;
        d.kout[0] = k;
    }
    __syncthreads();
    const int k = s_k;
    for (int r = tid; r < d.kmax; r += NT) d.sigma[r] = r < k ? sig[perm[r]] : 0.0;
    // left vectors of the processed matrix: A's columns / sigma (m rows);
    // right vectors: V's columns (n rows); for G^T they are G's Y and X
    double *lv = tr ? d.y : d.x, *rv = tr ? d.x : d.y;
    const int ldl = tr ? d.ldy : d.ldx, ldr = tr ? d.ldx : d.ldy;
    for (int e = tid; e < d.kmax * NMAX; e += NT) {
        const int i = e % NMAX, r = e / NMAX;
        const int p = r < k ? perm[r] : 0;
        if (i < m) lv[i + (size_t)r * ldl] = r < k ? A[p * LD + i] / sig[p] : 0.0;
        if (i < n) rv[i + (size_t)r * ldr] = r < k ? V[p * LD + i] : 0.0;
    }
}

// Cores of at most nmax rows and columns (nmax in {16, 32, 64}).
int launch_core_svd(int nmax, const SvdDesc *descs, int count, void *stream)
{
    if (count <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    if (nmax == 16)
        hipLaunchKernelGGL(lrbg_core_svd_kernel<16>, dim3(count), dim3(64), 0, s, descs, count);
    else if (nmax == 32)
        hipLaunchKernelGGL(lrbg_core_svd_kernel<32>, dim3(count), dim3(128), 0, s, descs, count);
    else if (nmax == 64)
        hipLaunchKernelGGL(lrbg_core_svd_kernel<64>, dim3(count), dim3(256), 0, s, descs, count);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int svd_max_dim() { return kSvdMax; }

}  // namespace lrbg
