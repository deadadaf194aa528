// Bosonic exchange spring energy (the bosonic fix of Sec. III.C; the
// recursion of Hirshberg et al. 2019, evaluated in O(N^2) like Feldman and
// Hirshberg's algorithm, both cited by the paper).  N identical
// particles, P beads; the springs inside each particle's ring are the
// distinguishable ones, and the link from bead P-1 of a particle to bead 0 of
// the next is summed over exchange cycles by
//   exp(-beta_n V[n]) = (1/n) sum_{k=1..n} exp(-beta_n (E[n,k] + V[n-k])),
// E[n,k] the single ring through particles n-k..n-1 (0-based), V[0] = 0.
// One block: the recursion is sequential in n and parallel in k; its
// gradient comes from the adjoints of the same recursion (each V[n] is a
// soft minimum with weights w[n,k] that sum to one), recomputed rather than
// stored, so the block holds O(N) values.
#include "pimd_internal.h"
#include "pimd_device.h"

namespace pimd {

namespace {

constexpr int kBosonMax = 512;   // particles per call (LDS-resident end beads)

struct BosonLds {
    double e0[kBosonMax * 3];    // bead 0 of each particle
    double el[kBosonMax * 3];    // bead P-1
    double sint[kBosonMax + 1];  // prefix sums of the particles' inner ring energies
    double schain[kBosonMax + 1];// prefix sums of the links l -> l+1
    double V[kBosonMax + 1];
    double adj[kBosonMax + 1];
    double wsuf[kBosonMax + 1];  // one n's ring weights, then their suffix sums over k
    double chain[kBosonMax];     // probability of the chain link l -> l+1
    double red[64];
};

__device__ __forceinline__ double link_e(const BosonLds &s, double kspring, int l, int l2)
{
    double e = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double dd = s.e0[l2 * 3 + d] - s.el[l * 3 + d];
        e += dd * dd;
    }
    return kspring * e;
}

// E[n,k]: inner rings of particles n-k..n-1, the chain links between them,
// and the closing link from n-1 back to n-k
__device__ __forceinline__ double ring_e(const BosonLds &s, double kspring, int n, int k)
{
    return (s.sint[n] - s.sint[n - k]) + (s.schain[n - 1] - s.schain[n - k]) +
           link_e(s, kspring, n - 1, n - k);
}

__device__ double block_min1(double v, double *red)
{
    constexpr int NW = kBlock / 64;
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    if ((t & 63) == 0) red[w] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int u = 1; u < NW; ++u) v = fmin(v, red[u]);
    __syncthreads();
    return v;
}

__device__ double block_sum1(double v, double *red)
{
    double a[1] = {v};
    block_sum<1>(a, red);
    __syncthreads();
    return a[0];
}

// x, f: [P][N][3] (bead, particle, dim); prob: [N][N]; out[0] = V_B
__global__ __launch_bounds__(kBlock) void k_boson_spring(const double *x, int N, int P,
                                                         double kspring, double beta_n,
                                                         double *f, double *prob, double *out)
{
    __shared__ BosonLds s;
    const int t = threadIdx.x;
    auto X = [&](int j, int l, int d) { return x[((size_t)j * N + l) * 3 + d]; };
    for (int e = t; e < N * 3; e += kBlock) {
        const int l = e / 3, d = e - l * 3;
        s.e0[e] = X(0, l, d);
        s.el[e] = X(P - 1, l, d);
    }
    // inner ring energies, then both prefix sums in index order (thread 0)
    for (int l = t; l < N; l += kBlock) {
        double e = 0.0;
        for (int j = 0; j + 1 < P; ++j)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double dd = X(j + 1, l, d) - X(j, l, d);
                e += dd * dd;
            }
        s.sint[l + 1] = kspring * e;
    }
    __syncthreads();
    if (t == 0) {
        s.sint[0] = 0.0;
        for (int l = 1; l <= N; ++l) s.sint[l] += s.sint[l - 1];
        s.schain[0] = 0.0;
        for (int l = 1; l < N; ++l) s.schain[l] = s.schain[l - 1] + link_e(s, kspring, l - 1, l);
        s.schain[N] = s.schain[N - 1];
        s.V[0] = 0.0;
    }
    __syncthreads();
    // forward: V[n] as a soft minimum over k, stabilized by the minimum
    for (int n = 1; n <= N; ++n) {
        double lo = INFINITY;
        for (int k = 1 + t; k <= n; k += kBlock) lo = fmin(lo, ring_e(s, kspring, n, k) + s.V[n - k]);
        lo = block_min1(lo, s.red);
        double sum = 0.0;
        for (int k = 1 + t; k <= n; k += kBlock)
            sum += exp(-beta_n * (ring_e(s, kspring, n, k) + s.V[n - k] - lo));
        sum = block_sum1(sum, s.red);
        if (t == 0) s.V[n] = lo - log(sum / (double)n) / beta_n;
        __syncthreads();
    }
    // backward: adj[n] = dV[N]/dV[n]; weights recomputed from E and V
    for (int e = t; e <= N; e += kBlock) s.adj[e] = (e == N) ? 1.0 : 0.0;
    __syncthreads();
    for (int n = N; n >= 1; --n) {
        const double an = s.adj[n];
        for (int k = 1 + t; k <= n; k += kBlock) {
            const double w = exp(-beta_n * (ring_e(s, kspring, n, k) + s.V[n - k] - s.V[n])) / (double)n;
            s.adj[n - k] += an * w;     // distinct k: distinct targets
        }
        __syncthreads();
    }
    // link probabilities.  Ring (n, k) carries q[n,k] = adj[n] w[n,k]: its
    // closing link n-1 -> n-k takes q[n,k], and each chain link l -> l+1 with
    // n-k <= l <= n-2 takes it too, so the chain link l gets, from each n,
    // the suffix sum over k >= n-l of q[n,k]: one block scan per n, O(N^2)
    // in all.
    for (int e = t; e < N * N; e += kBlock) prob[e] = 0.0;
    for (int l = t; l < N; l += kBlock) s.chain[l] = 0.0;
    __syncthreads();
    constexpr int KT = (kBosonMax + kBlock - 1) / kBlock;   // k per thread
    for (int n = 1; n <= N; ++n) {
        for (int k = 1 + t; k <= n; k += kBlock) {
            const double q = s.adj[n] *
                             exp(-beta_n * (ring_e(s, kspring, n, k) + s.V[n - k] - s.V[n])) / (double)n;
            prob[(size_t)(n - 1) * N + (n - k)] = q;    // one (n, k) per entry
            s.wsuf[k] = q;
        }
        __syncthreads();
        // suffix sums over k = 1..n (Hillis-Steele, in place)
        for (int off = 1; off < n; off <<= 1) {
            double add[KT];
#pragma unroll
            for (int u = 0; u < KT; ++u) {
                const int k = 1 + t + u * kBlock;
                add[u] = (k <= n && k + off <= n) ? s.wsuf[k + off] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < KT; ++u) {
                const int k = 1 + t + u * kBlock;
                if (k <= n) s.wsuf[k] += add[u];
            }
            __syncthreads();
        }
        // chain link l (l <= n-2) collects the rings with k >= n-l
        for (int l = t; l + 2 <= n; l += kBlock) s.chain[l] += s.wsuf[n - l];
        __syncthreads();
    }
    for (int l = t; l + 1 < N; l += kBlock) prob[(size_t)l * N + l + 1] = s.chain[l];
    __threadfence_block();
    __syncthreads();
    // link forces, one thread per particle: its last bead pulled toward the
    // first beads it links to, its first bead toward the last beads linking
    // to it
    for (int l = t; l < N; l += kBlock) {
        double gl[3] = {0.0, 0.0, 0.0}, g0[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < N; ++m) {
            const double qo = prob[(size_t)l * N + m], qi = prob[(size_t)m * N + l];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                gl[d] += 2.0 * kspring * qo * (s.e0[m * 3 + d] - s.el[l * 3 + d]);
                g0[d] -= 2.0 * kspring * qi * (s.e0[l * 3 + d] - s.el[m * 3 + d]);
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[((size_t)(P - 1) * N + l) * 3 + d] += gl[d];
            f[((size_t)0 * N + l) * 3 + d] += g0[d];
        }
    }
    if (t == 0) out[0] = s.V[N];
}

// The springs inside every particle's ring (weight one: each particle lies
// on one cycle), one thread per bead; this sets f, and k_boson_spring then
// adds the links.
__global__ __launch_bounds__(kBlock) void k_boson_inner(const double *x, int N, int P,
                                                        double kspring, double *f)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= N * P) return;
    const int j = e / N, l = e - j * N;
    auto X = [&](int jj, int d) { return x[((size_t)jj * N + l) * 3 + d]; };
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double g = 0.0;
        if (j + 1 < P) g += 2.0 * kspring * (X(j + 1, d) - X(j, d));
        if (j > 0) g -= 2.0 * kspring * (X(j, d) - X(j - 1, d));
        f[((size_t)j * N + l) * 3 + d] = g;
    }
}

// The potential's forces added to the springs': a harmonic trap
// U = 1/2 m mvv2e omega^2 |x|^2 per bead (kk = m mvv2e omega^2), and each
// bead's U for the energies.
__global__ __launch_bounds__(kBlock) void k_boson_trap(const double *x, int N, int P, double kk,
                                                       double *f, double *ubead)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= N * P) return;
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double xv = x[(size_t)e * 3 + d];
        f[(size_t)e * 3 + d] -= kk * xv;
        r2 += xv * xv;
    }
    ubead[e] = 0.5 * kk * r2;
}

// B(dt/2) A(dt/2) O(dt) A(dt/2) per bead velocity component (the opening of a
// step), or B(dt/2) alone (the closing): Cartesian, every bead with the same
// c1 (Eq. D3), noise of counter (particle, bead, step, 0).
__global__ __launch_bounds__(kBlock) void k_boson_update(double *x, double *v, const double *f,
                                                         int N, int P, double h, double im,
                                                         double c1, double c2, double sigma,
                                                         unsigned long long seed,
                                                         unsigned long long step, int opening,
                                                         int thermo)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= N * P) return;
    const int j = e / N, l = e - j * N;
    double z[3] = {0.0, 0.0, 0.0};
    if (opening && thermo)
        gauss3(seed, (unsigned long long)l, (unsigned long long)j, step, z, 0ULL);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const size_t q = (size_t)e * 3 + d;
        double vv = v[q] + h * f[q] * im;
        if (opening) {
            double xx = x[q] + h * vv;
            vv = c1 * vv + c2 * sigma * z[d];
            x[q] = xx + h * vv;
        }
        v[q] = vv;
    }
}

}  // namespace

int boson_max() { return kBosonMax; }

void launch_boson_forces(const double *x, int N, int P, double kspring, double beta_n, double kk,
                         double *f, double *prob, double *ubead, double *vb, hipStream_t st)
{
    launch_boson_spring(x, N, P, kspring, beta_n, f, prob, vb, st);
    hipLaunchKernelGGL(k_boson_trap, dim3((N * P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, x, N,
                       P, kk, f, ubead);
}

void launch_boson_update(double *x, double *v, const double *f, int N, int P, double h, double im,
                         double c1, double c2, double sigma, unsigned long long seed,
                         unsigned long long step, int opening, int thermo, hipStream_t st)
{
    hipLaunchKernelGGL(k_boson_update, dim3((N * P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, x,
                       v, f, N, P, h, im, c1, c2, sigma, seed, step, opening, thermo);
}

void launch_boson_spring(const double *x, int N, int P, double kspring, double beta_n, double *f,
                         double *prob, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_boson_inner, dim3((N * P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, x,
                       N, P, kspring, f);
    hipLaunchKernelGGL(k_boson_spring, dim3(1), dim3(kBlock), 0, st, x, N, P, kspring, beta_n, f,
                       prob, out);
}

}  // namespace pimd
