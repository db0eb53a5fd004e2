// Kernels on the stored band as a whole.  Equal time blocks of an equidistant grid (eq.
// (relationAtildeBlock), Section 5.1): the blocks that equal_block_source maps to an integrated
// block are filled by copying that block's stored values, so an equidistant assembly integrates
// O(N) node blocks instead of O(N^2).  The deterministic assembly's scale and conversion.
#include "tdbem_internal.hpp"

namespace tdbem {

// One workgroup per (time row k, vertex tile t); lane = column j % 64 of the tile, the four waves
// walk its rows.  Every write goes to a copied block and every read to an integrated one, so the
// workgroups are independent.  The band of a copied pair (l, j) and the band of its source hold
// the same trial indices up to the rounding of the kernel supports: a source slot outside the
// source's band stands for a value that is zero.
template <typename V>
__global__ void __launch_bounds__(256) k_block_copy(BandView b, V* __restrict__ val)
{
    const int64_t q = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    if (q >= (int64_t)b.N * b.nt) return;
    const int k = (int)(q / b.nt);
    const int64_t t = q - (int64_t)k * b.nt;
    const int kn = k / b.p1, m2 = k - kn * b.p1;
    if (kn < 1 || kn > b.nodes - 2) return;     // rows of the first and last node are integrated
    const int B = b.B[q];
    if (B == 0) return;
    int tl = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(tl + 1) * (tl + 2) / 2 <= t) ++tl;
    while ((int64_t)tl * (tl + 1) / 2 > t) --tl;
    const int tj = (int)(t - (int64_t)tl * (tl + 1) / 2);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j = (int64_t)tj * kBT + lane;
    const int16_t* il = b.ilo + q * (kBT * kBT);
    for (int lr = wave; lr < kBT; lr += 4) {
        const int64_t l = (int64_t)tl * kBT + lr;
        if (l >= b.M || j > l) continue;
        const int e = lr * kBT + lane;
        const int ilo = il[e];
        V* dst = val + b.voff[q] + (int64_t)lr * B * kBT + lane;
        for (int s = 0; s < B; ++s) {
            const int i = ilo + s;
            if (i >= b.N) break;
            const int in = i / b.p1;
            int sk, si;
            if (!equal_block_source(b.nodes, kn, in, sk, si)) continue;
            const int64_t qs = (int64_t)(sk * b.p1 + m2) * b.nt + t;
            const int Bs = b.B[qs];
            const int ss = si * b.p1 + (i - in * b.p1) - (int)b.ilo[qs * (kBT * kBT) + e];
            V v = V(0);
            if (ss >= 0 && ss < Bs) v = val[b.voff[qs] + ((int64_t)lr * Bs + ss) * kBT + lane];
            dst[(int64_t)s * kBT] = v;
        }
    }
}

void launch_block_copy(BandView band, double* val, float* valf, hipStream_t s)
{
    const int64_t n = (int64_t)band.N * band.nt;
    if (n <= 0) return;
    const int64_t gx = n < 65536 ? n : 65536;
    dim3 grid((unsigned)gx, (unsigned)((n + gx - 1) / gx));
    if (valf)
        hipLaunchKernelGGL(k_block_copy<float>, grid, dim3(256), 0, s, band, valf);
    else
        hipLaunchKernelGGL(k_block_copy<double>, grid, dim3(256), 0, s, band, val);
}

// Largest |value| of the storage: a non-negative double orders like its bit pattern, so the
// maximum is an integer atomic max over the patterns.
__global__ void __launch_bounds__(256) k_absmax(const double* __restrict__ val, int64_t n,
                                                unsigned long long* __restrict__ out)
{
    double m = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(val[s]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Fixed-point integers of scale 2^e (two's complement in the 8 bytes of each value) to doubles:
// one rounding to 53 bits, then an exact scaling.
__global__ void __launch_bounds__(256) k_fixed_to_double(double* __restrict__ val, int64_t n, int e)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const long long q = __double_as_longlong(val[s]);
    val[s] = ldexp((double)q, -e);
}

void launch_absmax(const double* val, int64_t n, double* out, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t blocks = (n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384;
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, s, val, n,
                       reinterpret_cast<unsigned long long*>(out));
}

void launch_fixed_to_double(double* val, int64_t n, int e, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fixed_to_double, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, val, n, e);
}

}  // namespace tdbem
