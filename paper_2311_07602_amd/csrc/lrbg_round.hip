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
// 4 or 8 lanes per pair.  For a pair with alpha = |a_p|^2, beta = |a_q|^2,
// gamma = a_p . a_q the rotation zeta = (beta - alpha) / (2 gamma),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t,
// a_p <- c a_p - s a_q, a_q <- s a_p + c a_q makes the pair orthogonal.
#include "lrbg_tiles.h"

namespace lrbg {

constexpr int kSvdMax = 64;    // m, n <= 64
constexpr int kSvdSweeps = 40;

// Sum over the LPP lanes of a pair (aligned groups of 4 or 8 lanes) with
// DPP lane swaps: xor 1 and xor 2 inside a quad, then the half-row mirror
// (lane i <-> 7 - i) joins the two quads of an 8-lane group.  Every level
// adds the same two values in either order, so all lanes of the group end
// with the identical sum.
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double x)
{
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int LPP>
__device__ __forceinline__ double pair_sum(double x)
{
    static_assert(LPP == 4 || LPP == 8, "4 or 8 lanes per pair");
    x += dpp_swap<0xB1>(x);              // quad_perm [1,0,3,2]
    x += dpp_swap<0x4E>(x);              // quad_perm [2,3,0,1]
    if constexpr (LPP == 8) x += dpp_swap<0x141>(x);   // row_half_mirror
    return x;
}

// One core per workgroup of NMAX / 2 pairs x LPP lanes.  G and V live in LDS
// by tournament position, not by column: position x sits in slot x (stride
// LD, zero-padded to NMAX rows), so the pair that owns positions pr and
// N-1-pr reads the same two slots at every step, and each step writes the
// rotated columns to the slots their positions take next (the circle
// method: position 0 stays, the column at position x >= 2 moves to x - 1 and
// the one at 1 moves to N - 1).  Rows are placed so that the LPP lanes of
// 32 / LPP consecutive slots cover distinct banks (reads never conflict; a
// write meets at most one other pair's lanes, at the wrap-around slot):
// either row i of slot x sits at i ^ (LPP (x mod 32 / LPP)) in an unpadded
// slot, or, where that would leave the slot, slots are padded to a stride
// that is an odd multiple of LPP.  The rotation is symmetric in the two columns (with
// their roles swapped zeta, t and s change sign and the rotated pair is the
// same), so which of the two is "p" does not matter.  Cores up to 32 wide
// take one wave, whose reads of a step complete before its writes; wider
// ones separate the two with a barrier.
template <int NMAX, int LPP, int CPW>
__global__ void __launch_bounds__(NMAX / 2 * LPP * CPW)
lrbg_core_svd_kernel(const SvdDesc *__restrict__ descs, int count)
{
    constexpr int NT = NMAX / 2 * LPP, RPL = NMAX / LPP;   // threads per core
    static_assert(CPW == 1 || NT * CPW <= 64, "several cores per workgroup only within one wave");
    constexpr bool SWZ = 32 / LPP <= RPL;
    constexpr int LD = SWZ ? NMAX : NMAX + LPP;
    static_assert(NMAX % (2 * LPP) == 0, "a padded stride must be an odd multiple of LPP");
    // element (slot x, row i)
    auto at = [](int x, int i) { return x * LD + (SWZ ? (i ^ (LPP * (x & (32 / LPP - 1)))) : i); };
    __shared__ double A_[CPW][NMAX * LD];
    __shared__ double V_[CPW][NMAX * LD];
    __shared__ double sig_[CPW][NMAX];
    __shared__ int32_t perm_[CPW][NMAX];
    __shared__ int32_t s_k_[CPW];
    // CPW cores per workgroup, NT threads each (a trailing workgroup may hold
    // fewer live cores; every thread still takes part in the barriers)
    const int cw = CPW == 1 ? 0 : (int)threadIdx.x / NT, tid = CPW == 1 ? (int)threadIdx.x : (int)threadIdx.x % NT;
    const int t = blockIdx.x * CPW + cw;
    const bool live = CPW == 1 || t < count;   // one core per workgroup: the grid is the count
    double *A = A_[cw], *V = V_[cw], *sig = sig_[cw];
    int32_t *perm = perm_[cw], &s_k = s_k_[cw];
    SvdDesc d{};
    if (CPW == 1)
        d = descs[t];
    else if (live)
        d = descs[t];
    const bool tr = d.m < d.n;                     // work on G^T
    const int m = tr ? d.n : d.m, n = tr ? d.m : d.n;

    // column p starts in slot p
    for (int e = tid; e < NMAX * NMAX; e += NT) {
        const int i = e % NMAX, p = e / NMAX;
        double v = 0.0;
        if (i < m && p < n) v = tr ? d.g[p + (size_t)i * d.ldg] : d.g[i + (size_t)p * d.ldg];
        A[at(p, i)] = v;
        V[at(p, i)] = (i == p) ? 1.0 : 0.0;
    }
    __syncthreads();

    const int N = (n + 1) & ~1;                    // a zero column pads odd n
    const int pairs = N / 2, pr = tid / LPP, ll = tid % LPP;
    const int sa = pr, sb = N - 1 - pr;            // this pair's slots
    const int na = sa == 0 ? 0 : (sa == 1 ? N - 1 : sa - 1);
    const int nb = sb == 0 ? 0 : (sb == 1 ? N - 1 : sb - 1);
    const bool active = pr < pairs;
    // uniform over the workgroup: with several cores the sweeps continue
    // until none of them rotates (a converged or empty core just moves its
    // columns)
    for (int sweep = 0; sweep < kSvdSweeps && (CPW > 1 || N >= 2); ++sweep) {
        int rotated = 0;
        for (int step = 0; step < N - 1; ++step) {
            double x[RPL], y[RPL], vx[RPL], vy[RPL];
            if (active) {
#pragma unroll
                for (int j = 0; j < RPL; ++j) {
                    x[j] = A[at(sa, ll + LPP * j)];
                    y[j] = A[at(sb, ll + LPP * j)];
                    vx[j] = V[at(sa, ll + LPP * j)];
                    vy[j] = V[at(sb, ll + LPP * j)];
                }
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int j = 0; j < RPL; ++j) {
                    al += x[j] * x[j];
                    be += y[j] * y[j];
                    ga += x[j] * y[j];
                }
                al = pair_sum<LPP>(al);
                be = pair_sum<LPP>(be);
                ga = pair_sum<LPP>(ga);
                if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = rsqrt(1.0 + tt * tt), s = c * tt;   // 1 / sqrt, one call
#pragma unroll
                    for (int j = 0; j < RPL; ++j) {
                        const double x0 = x[j], y0 = y[j], v0 = vx[j], w0 = vy[j];
                        x[j] = c * x0 - s * y0;
                        y[j] = s * x0 + c * y0;
                        vx[j] = c * v0 - s * w0;
                        vy[j] = s * v0 + c * w0;
                    }
                    rotated = 1;
                }
            }
            if constexpr (NT * CPW > 64) __syncthreads();   // every wave has read its slots
            if (active) {
#pragma unroll
                for (int j = 0; j < RPL; ++j) {
                    A[at(na, ll + LPP * j)] = x[j];
                    A[at(nb, ll + LPP * j)] = y[j];
                    V[at(na, ll + LPP * j)] = vx[j];
                    V[at(nb, ll + LPP * j)] = vy[j];
                }
            }
            // One wave: its LDS accesses execute in issue order, so the next
            // step's reads see these writes; only the compiler must not
            // reorder them.  Several waves: a workgroup barrier.
            if constexpr (NT * CPW <= 64)
                __builtin_amdgcn_wave_barrier();
            else
                __syncthreads();
        }
        if (!__syncthreads_or(rotated)) break;
    }

    // singular values by slot (the pad column has sigma 0), descending order
    // (ties by slot), truncation rank
    if (tid < N) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += A[at(tid, i)] * A[at(tid, i)];
        sig[tid] = sqrt(s2);
    }
    __syncthreads();
    if (tid < N) {
        int rank = 0;
        for (int j = 0; j < N; ++j) rank += (sig[j] > sig[tid]) || (sig[j] == sig[tid] && j < tid);
        perm[rank] = tid;
    }
    __syncthreads();
    if (tid == 0 && live) {
        const double smax = n > 0 ? sig[perm[0]] : 0.0;
        int k = 0;
        while (k < n && k < d.kmax && smax > 0.0 && sig[perm[k]] > d.tol * smax) ++k;
        s_k = k;
        d.kout[0] = k;
    }
    __syncthreads();
    const int k = s_k;
    for (int r = tid; r < d.kmax; r += NT) d.sigma[r] = r < k ? sig[perm[r]] : 0.0;
    // left vectors of the processed matrix: A's slots / sigma (m rows);
    // right vectors: V's slots (n rows); for G^T they are G's Y and X
    double *lv = tr ? d.y : d.x, *rv = tr ? d.x : d.y;
    const int ldl = tr ? d.ldy : d.ldx, ldr = tr ? d.ldx : d.ldy;
    for (int e = tid; e < d.kmax * NMAX; e += NT) {
        const int i = e % NMAX, r = e / NMAX;
        const int p = r < k ? perm[r] : 0;
        if (i < m) lv[i + (size_t)r * ldl] = r < k ? A[at(p, i)] / sig[p] : 0.0;
        if (i < n) rv[i + (size_t)r * ldr] = r < k ? V[at(p, i)] : 0.0;
    }
}

// Cores of at most nmax rows and columns (nmax in {16, 32, 64}).
int launch_core_svd(int nmax, const SvdDesc *descs, int count, void *stream)
{
    if (count <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    if (nmax == 16)   // two cores per wave, one per half
        hipLaunchKernelGGL((lrbg_core_svd_kernel<16, 4, 2>), dim3((count + 1) / 2), dim3(64), 0, s, descs, count);
    else if (nmax == 32)
        hipLaunchKernelGGL((lrbg_core_svd_kernel<32, 4, 1>), dim3(count), dim3(64), 0, s, descs, count);
    else if (nmax == 64)
        hipLaunchKernelGGL((lrbg_core_svd_kernel<64, 8, 1>), dim3(count), dim3(256), 0, s, descs, count);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int svd_max_dim() { return kSvdMax; }

}  // namespace lrbg
