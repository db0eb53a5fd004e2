// Learned variable preconditioner for FGMRES (not part of the paper) and the transposed block
// matvec its training needs.
//
// The network acts on the space-time graph of the block partition of eq. (A): node n = k*M + j
// is the unknown of (b_k, phi_j).  Every node carries 64 float32 channels.  One layer forms the
// 256 features [h(k,j), mean of h(k,j') over the mesh neighbours j' of j, h(k-1,j), h(k+1,j)]
// (zero outside the time range), multiplies them by a 64 x 256 bfloat16 weight matrix with
// float32 accumulation, adds a float32 bias and updates h += relu(u).  The input layer maps
// [v/s, h_k/hbar, h_{k+1}/hbar] to 64 channels, the output is z = s * (h . wout), with s the root
// mean square of v.  Parameters are kept as float32 master copies (Adam) and used as bfloat16.
#include "tdbem_internal.hpp"

namespace tdbem {

constexpr int kH = kLpHidden;          // channels per node
constexpr int kTile = 64;              // nodes per tile of the dense layer kernels
constexpr int kPad = kH + 4;           // LDS row pitch (floats)
constexpr int kChunk = 256;            // nodes per workgroup of the reduction kernels

__device__ inline float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline uint16_t float_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);     // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__global__ void __launch_bounds__(256) k_lp_round(int64_t P, const float* __restrict__ p, uint16_t* __restrict__ q)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < P) q[s] = float_to_bf16(p[s]);
}

// Load the 64 x 64 feature block `part` of the nodes [n0, n0 + 64) into LDS:
// part 0: h, 1: neighbour mean of h, 2: h of the previous time block, 3: of the next one.
__device__ inline void load_features(float (*xs)[kPad], const LpGraph& g, int64_t n, int64_t n0, int part,
                                     const float* __restrict__ h)
{
    const int r = threadIdx.x >> 2;            // node of the tile
    const int c0 = (threadIdx.x & 3) * 16;     // 16 channels
    const int64_t node = n0 + r;
    float4 a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (node < n) {
        const int k = (int)(node / g.M), j = (int)(node - (int64_t)k * g.M);
        if (part == 0 || (part == 2 && k > 0) || (part == 3 && k + 1 < g.N)) {
            const int64_t src = part == 0 ? node : (part == 2 ? node - g.M : node + g.M);
            const float4* hp = reinterpret_cast<const float4*>(h + src * kH + c0);
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = hp[q];
        } else if (part == 1) {
            const int b = g.ptr[j], e = g.ptr[j + 1];
            for (int u = b; u < e; ++u) {
                const float4* hp = reinterpret_cast<const float4*>(h + ((int64_t)k * g.M + g.idx[u]) * kH + c0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float4 w = hp[q];
                    a[q].x += w.x; a[q].y += w.y; a[q].z += w.z; a[q].w += w.w;
                }
            }
            const float inv = e > b ? 1.0f / (float)(e - b) : 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) { a[q].x *= inv; a[q].y *= inv; a[q].z *= inv; a[q].w *= inv; }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<float4*>(&xs[r][c0 + 4 * q]) = a[q];
}

// LDS wt[c][o] = W[o][part*64 + c] (transposed block).
__device__ inline void load_weights_t(float (*wt)[kPad], const uint16_t* __restrict__ W, int part)
{
    const int o = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    const uint16_t* src = W + o * (4 * kH) + part * kH + c0;
#pragma unroll
    for (int q = 0; q < 16; ++q) wt[c0 + q][o] = bf16_to_float(src[q]);
}

// H0[n][c] = bin[c] + Win[c] . [v_n / s, f1_k, f2_k]
__global__ void __launch_bounds__(256)
k_lp_input(int64_t n, LpGraph g, const double* __restrict__ v, const double* __restrict__ sc,
           const uint16_t* __restrict__ Win,
           const float* __restrict__ bin, float* __restrict__ H0)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * kH) return;
    const int64_t node = s / kH;
    const int c = (int)(s - node * kH);
    const int k = (int)(node / g.M);
    const float x0 = (float)(v[node] * sc[1]);
    const float f1 = g.feat[2 * k], f2 = g.feat[2 * k + 1];
    float a = bin[c];
    a = fmaf(bf16_to_float(Win[3 * c + 0]), x0, a);
    a = fmaf(bf16_to_float(Win[3 * c + 1]), f1, a);
    a = fmaf(bf16_to_float(Win[3 * c + 2]), f2, a);
    H0[s] = a;
}

// One message-passing layer on a tile of 64 nodes, U = X W^T + b, Hout = Hin + relu(U), with the
// 64 x 256 x 64 product on the matrix cores (v_mfma_f32_16x16x32_bf16): wave w forms the output
// channels 16 w .. 16 w + 15 of the tile's 64 nodes as four 16 x 16 blocks over K = 256.  A float32
// feature x enters as three bfloat16 parts hi + mid + lo (8 + 8 + 8 significant bits, x - hi - mid -
// lo below 2^-24 |x|); each part times a bfloat16 weight is exact in float32 and the products are
// accumulated in float32, so the layer keeps float32 accuracy.
// Fragments: lane l holds A[m = l % 16][k = 8 (l / 16) + i], B[k = 8 (l / 16) + i][n = l % 16] for
// i < 8, and D[m = 4 (l / 16) + r][n = l % 16] for r < 4.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

__global__ void __launch_bounds__(256)
k_lp_layer(int64_t n, LpGraph g, const float* __restrict__ Hin, const uint16_t* __restrict__ W,
                const float* __restrict__ bias, float* __restrict__ Hout, float* __restrict__ U)
{
    __shared__ float xs[kTile][kPad];
    const int64_t n0 = (int64_t)blockIdx.x * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    floatx4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int part = 0; part < 4; ++part) {
        load_features(xs, g, n, n0, part, Hin);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kH; ks += 32) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(W + (16 * wave + col) * (4 * kH) + part * kH + ks + 8 * kq);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float* xr = &xs[16 * t + col][ks + 8 * kq];
                bf16x8 hi, mid, lo;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float x = xr[i];
                    const __bf16 h = (__bf16)x;
                    const float r1 = x - (float)h;
                    const __bf16 m = (__bf16)r1;
                    hi[i] = h;
                    mid[i] = m;
                    lo[i] = (__bf16)(r1 - (float)m);
                }
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, b, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mid, b, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int ch = 16 * wave + col;
    const float bc = bias[ch];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t node = n0 + 16 * t + 4 * kq + r;
            if (node >= n) continue;
            const float u = acc[t][r] + bc;
            Hout[node * kH + ch] = Hin[node * kH + ch] + fmaxf(u, 0.f);
            if (U) U[node * kH + ch] = u;
        }
}

// z_n = s * sum_c wout[c] H[n][c]
__global__ void __launch_bounds__(256)
k_lp_output(int64_t n, const float* __restrict__ H, const uint16_t* __restrict__ wout, const double* __restrict__ sc,
            double* __restrict__ z)
{
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= n) return;
    const float4* hp = reinterpret_cast<const float4*>(H + node * kH);
    float a = 0.f;
#pragma unroll
    for (int q = 0; q < kH / 4; ++q) {
        const float4 h = hp[q];
        a = fmaf(h.x, bf16_to_float(wout[4 * q + 0]), a);
        a = fmaf(h.y, bf16_to_float(wout[4 * q + 1]), a);
        a = fmaf(h.z, bf16_to_float(wout[4 * q + 2]), a);
        a = fmaf(h.w, bf16_to_float(wout[4 * q + 3]), a);
    }
    z[node] = sc[0] * (double)a;
}

// Backward of the output: dH[n][c] = s dz_n wout[c]; partial[blk][c] = sum_n s dz_n H[n][c].
__global__ void __launch_bounds__(256)
k_lp_output_bwd(int64_t n, const float* __restrict__ H, const uint16_t* __restrict__ wout, const double* __restrict__ sc,
                const double* __restrict__ dz, float* __restrict__ dH, float* __restrict__ partial)
{
    __shared__ float red[4][kH];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * kChunk;
    const int64_t e = b + kChunk < n ? b + kChunk : n;
    const float w = bf16_to_float(wout[c]);
    float acc = 0.f;
    for (int64_t node = b + q; node < e; node += 4) {
        const float gz = (float)(sc[0] * dz[node]);
        dH[node * kH + c] = gz * w;
        acc = fmaf(gz, H[node * kH + c], acc);
    }
    red[q][c] = acc;
    __syncthreads();
    if (q == 0) partial[(int64_t)blockIdx.x * kH + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// Backward of a layer, part 1: DU = dH * [U > 0] and dX_p = DU W_p (the 4 feature blocks), the
// products on the matrix cores as in k_lp_layer (DU split into three bfloat16 parts; the
// weights are bfloat16 values, exact in either format).  Wave w forms the channels 16 w .. 16 w +
// 15 of every part for the tile's 64 nodes.
__global__ void __launch_bounds__(256)
k_lp_layer_bwd_dx(int64_t n, const float* __restrict__ U, const float* __restrict__ dH,
                  const uint16_t* __restrict__ W, float* __restrict__ DU, float* __restrict__ dX)
{
    __shared__ float ds[kTile][kPad];
    __shared__ float wt[kH][kPad];
    const int64_t n0 = (int64_t)blockIdx.x * kTile;
    {
        const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
        const int64_t node = n0 + r;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float d = 0.f;
            if (node < n) {
                const float u = U[node * kH + c0 + q];
                d = u > 0.f ? dH[node * kH + c0 + q] : 0.f;
                DU[node * kH + c0 + q] = d;
            }
            ds[r][c0 + q] = d;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int c = 16 * wave + col;
    for (int part = 0; part < 4; ++part) {
        load_weights_t(wt, W, part);
        __syncthreads();
        floatx4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kH; ks += 32) {
            bf16x8 b;
#pragma unroll
            for (int i = 0; i < 8; ++i) b[i] = (__bf16)wt[c][ks + 8 * kq + i];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float* dr = &ds[16 * t + col][ks + 8 * kq];
                bf16x8 hi, mid, lo;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float x = dr[i];
                    const __bf16 h = (__bf16)x;
                    const float r1 = x - (float)h;
                    const __bf16 m = (__bf16)r1;
                    hi[i] = h;
                    mid[i] = m;
                    lo[i] = (__bf16)(r1 - (float)m);
                }
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, b, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(mid, b, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, b, acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t node = n0 + 16 * t + 4 * kq + r;
                if (node < n) dX[((int64_t)part * n + node) * kH + c] = acc[t][r];
            }
        __syncthreads();
    }
}

// Backward of a layer, part 2: gradient with respect to the layer input,
// dHin(k,j) = dH(k,j) + dX_0(k,j) + sum_{j' ~ j} dX_1(k,j') / deg(j') + dX_2(k+1,j) + dX_3(k-1,j).
__global__ void __launch_bounds__(256)
k_lp_layer_bwd_gather(int64_t n, LpGraph g, const float* __restrict__ dH, const float* __restrict__ dX,
                      float* __restrict__ dHin)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * kH) return;
    const int64_t node = s / kH;
    const int c = (int)(s - node * kH);
    const int k = (int)(node / g.M), j = (int)(node - (int64_t)k * g.M);
    float a = dH[s] + dX[s];
    const float* dX1 = dX + n * kH;
    for (int u = g.ptr[j]; u < g.ptr[j + 1]; ++u) {
        const int jj = g.idx[u];
        const int deg = g.ptr[jj + 1] - g.ptr[jj];
        a += dX1[((int64_t)k * g.M + jj) * kH + c] / (float)deg;
    }
    if (k + 1 < g.N) a += dX[2 * n * kH + (node + g.M) * kH + c];
    if (k > 0) a += dX[3 * n * kH + (node - g.M) * kH + c];
    dHin[s] = a;
}

// Backward of a layer, part 3: weight and bias gradients over a chunk of 256 nodes,
// partial[blk][o*256 + p*64 + c] = sum_n DU[n][o] X_p[n][c], partial[blk][16384 + o] = sum_n DU[n][o].
__global__ void __launch_bounds__(256)
k_lp_layer_bwd_dw(int64_t n, LpGraph g, const float* __restrict__ Hin, const float* __restrict__ DU,
                  float* __restrict__ partial)
{
    __shared__ float xs[kTile][kPad];
    __shared__ float ds[kTile][kPad];
    const int tc = threadIdx.x & 15, to = threadIdx.x >> 4;
    float acc[4][4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[p][a][b] = 0.f;
    float bsum = 0.f;
    const int64_t cb = (int64_t)blockIdx.x * kChunk;
    for (int64_t n0 = cb; n0 < cb + kChunk && n0 < n; n0 += kTile) {
        __syncthreads();
        {
            const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
            const int64_t node = n0 + r;
#pragma unroll
            for (int q = 0; q < 16; ++q) ds[r][c0 + q] = node < n ? DU[node * kH + c0 + q] : 0.f;
        }
#pragma unroll
        for (int part = 0; part < 4; ++part) {
            load_features(xs, g, n, n0, part, Hin);
            __syncthreads();
            if (part == 0 && threadIdx.x < kH)
                for (int r = 0; r < kTile; ++r) bsum += ds[r][threadIdx.x];
#pragma unroll 4
            for (int r = 0; r < kTile; ++r) {
                const float4 d = *reinterpret_cast<const float4*>(&ds[r][4 * to]);
                const float4 x = *reinterpret_cast<const float4*>(&xs[r][4 * tc]);
                const float da[4] = {d.x, d.y, d.z, d.w};
                const float xb[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        // the feature block is selected at compile time by unrolling over part
                        if (part == 0) acc[0][a][b] = fmaf(da[a], xb[b], acc[0][a][b]);
                        else if (part == 1) acc[1][a][b] = fmaf(da[a], xb[b], acc[1][a][b]);
                        else if (part == 2) acc[2][a][b] = fmaf(da[a], xb[b], acc[2][a][b]);
                        else acc[3][a][b] = fmaf(da[a], xb[b], acc[3][a][b]);
                    }
            }
            __syncthreads();
        }
    }
    float* out = partial + (int64_t)blockIdx.x * (kH * 4 * kH + kH);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int a = 0; a < 4; ++a)
            *reinterpret_cast<float4*>(out + (4 * to + a) * (4 * kH) + p * kH + 4 * tc) =
                make_float4(acc[p][a][0], acc[p][a][1], acc[p][a][2], acc[p][a][3]);
    if (threadIdx.x < kH) out[kH * 4 * kH + threadIdx.x] = bsum;
}

// Backward of the input layer: partial[blk][c*3 + f] = sum_n dH0[n][c] x_f(n), partial[blk][192 + c]
// = sum_n dH0[n][c].
__global__ void __launch_bounds__(256)
k_lp_input_bwd(int64_t n, LpGraph g, const double* __restrict__ v, const double* __restrict__ sc,
               const float* __restrict__ dH0,
               float* __restrict__ partial)
{
    __shared__ float red[4][kH][4];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t b = (int64_t)blockIdx.x * kChunk;
    const int64_t e = b + kChunk < n ? b + kChunk : n;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int64_t node = b + q; node < e; node += 4) {
        const int k = (int)(node / g.M);
        const float d = dH0[node * kH + c];
        a0 = fmaf(d, (float)(v[node] * sc[1]), a0);
        a1 = fmaf(d, g.feat[2 * k], a1);
        a2 = fmaf(d, g.feat[2 * k + 1], a2);
        a3 += d;
    }
    red[q][c][0] = a0; red[q][c][1] = a1; red[q][c][2] = a2; red[q][c][3] = a3;
    __syncthreads();
    if (q == 0) {
        float* out = partial + (int64_t)blockIdx.x * (4 * kH);
        for (int f = 0; f < 3; ++f) out[3 * c + f] = red[0][c][f] + red[1][c][f] + red[2][c][f] + red[3][c][f];
        out[3 * kH + c] = red[0][c][3] + red[1][c][3] + red[2][c][3] + red[3][c][3];
    }
}

// grad[e] += sum_b partial[b][e], e < width
__global__ void __launch_bounds__(256)
k_lp_reduce(const float* __restrict__ partial, int nblk, int width, float* __restrict__ grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= width) return;
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += partial[(int64_t)b * width + e];
    grad[e] += a;
}

// Adam (Kingma and Ba 2015) on the float32 master parameters; refreshes the bfloat16 copy.
__global__ void __launch_bounds__(256)
k_lp_adam(int64_t P, float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ m,
          float* __restrict__ v2, float lr, float b1, float b2, float eps, float bc1, float bc2, float gscale,
          uint16_t* __restrict__ q)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P) return;
    const float g = grad[s] * gscale;
    const float mm = b1 * m[s] + (1.f - b1) * g;
    const float vv = b2 * v2[s] + (1.f - b2) * g * g;
    m[s] = mm;
    v2[s] = vv;
    const float np = p[s] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    p[s] = np;
    q[s] = float_to_bf16(np);
}

// Standard normal samples from a counter-based generator: SplitMix64 (Steele, Lea and Flood
// 2014) of (seed, stream, index) gives two uniforms, Box-Muller gives the normal value.
__device__ inline uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void __launch_bounds__(256)
k_lp_randn(int64_t n, uint64_t seed, uint64_t stream, double* __restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t base = splitmix64(seed ^ splitmix64(stream)) + 2 * (uint64_t)s;
    const uint64_t r1 = splitmix64(base), r2 = splitmix64(base + 1);
    const double u1 = ((double)(r1 >> 11) + 1.0) * 0x1.0p-53;     // (0, 1]
    const double u2 = (double)(r2 >> 11) * 0x1.0p-53;             // [0, 1)
    out[s] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586477 * u2);
}

// y = (x + neighbour mean of x) / 2 in every time block (a smoothing of training vectors).
__global__ void __launch_bounds__(256)
k_lp_smooth(int64_t n, LpGraph g, const double* __restrict__ x, double* __restrict__ y)
{
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= n) return;
    const int k = (int)(node / g.M), j = (int)(node - (int64_t)k * g.M);
    const int b = g.ptr[j], e = g.ptr[j + 1];
    double a = 0.0;
    for (int u = b; u < e; ++u) a += x[(int64_t)k * g.M + g.idx[u]];
    y[node] = 0.5 * x[node] + (e > b ? 0.5 * a / (e - b) : 0.0);
}

// x = A^T y for the whole operator.  Every block A_{k,i} is symmetric, so (A^T y)_i = sum_k
// A_{k,i} y_k: the stored value a = A_{k,i}(l, j), j <= l, adds a y_k(l) to x_i(j) and, off the
// diagonal, a y_k(j) to x_i(l).  Workgroup per (tile, k) as in the forward product.  The sums
// are collected in LDS over the tile's trial range [ibase, ibase + span) (LDS atomics; the row
// term is first summed over the wave when the band start is the same for the whole row) and
// added to x with one global atomic per (i, vertex); tiles with a wider range add straight to x.
constexpr int kSpanT = 40;

template <typename VT>
__global__ void __launch_bounds__(256)
k_matvec_tri_t(BandView band, const VT* __restrict__ val, const double* __restrict__ y, double* __restrict__ x)
{
    const int M = band.M, N = band.N;
    const int k = blockIdx.y;
    const int t = blockIdx.x;
    const int B = band.B[(int64_t)k * band.nt + t];
    if (B == 0) return;
    int tl = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tl + 1) * (tl + 2) / 2 <= t) ++tl;
    while (tl * (tl + 1) / 2 > t) --tl;
    const int tj = t - tl * (tl + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = tj * kBT + lane;
    const int16_t* __restrict__ il = band.ilo + ((int64_t)k * band.nt + t) * (kBT * kBT) + lane;
    const VT* __restrict__ vt = val + band.voff[(int64_t)k * band.nt + t] + lane;
    const double* __restrict__ yk = y + (int64_t)k * M;
    const double yj = j < M ? yk[j] : 0.0;
    __shared__ double s_dir[kSpanT][kBT];    // x_{ibase + r}(tj*64 + lane)
    __shared__ double s_mir[kSpanT][kBT];    // x_{ibase + r}(tl*64 + row)
    __shared__ int s_range[4][2];
    // trial range of the tile's stored slots
    int lo = 0x7fffffff, hi = -0x7fffffff;
    for (int m = 0; m < 16; ++m) {
        const int lr = wave + 4 * m;
        const int l = tl * kBT + lr;
        if (l < M && j <= l) {
            const int ib = il[lr * kBT];
            lo = min(lo, max(ib, 0));
            hi = max(hi, min(ib + B, N));
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) { s_range[wave][0] = lo; s_range[wave][1] = hi; }
    __syncthreads();
    const int ibase = min(min(s_range[0][0], s_range[1][0]), min(s_range[2][0], s_range[3][0]));
    const int itop = max(max(s_range[0][1], s_range[1][1]), max(s_range[2][1], s_range[3][1]));
    const int span = itop - ibase;
    const bool staged = span > 0 && span <= kSpanT;
    if (staged) {
        for (int e = threadIdx.x; e < span * kBT; e += 256) {
            s_dir[e / kBT][e % kBT] = 0.0;
            s_mir[e / kBT][e % kBT] = 0.0;
        }
    }
    __syncthreads();
    for (int m = 0; m < 16; ++m) {
        const int lr = wave + 4 * m;
        const int l = tl * kBT + lr;
        if (l >= M) break;
        const bool act = j <= l;
        const int ib = il[lr * kBT];
        const int slo = act ? (ib < 0 ? -ib : 0) : 0;
        const int shi = act ? (N - ib < B ? N - ib : B) : 0;
        const double yl = yk[l];
        const unsigned long long am = __ballot(act);
        if (am == 0) continue;
        const int first = __ffsll((long long)am) - 1;
        const int ib0 = __shfl(ib, first, 64);
        const bool uni = __ballot(act && ib != ib0) == 0;
        const int slo0 = ib0 < 0 ? -ib0 : 0, shi0 = N - ib0 < B ? N - ib0 : B;
        const VT* __restrict__ v = vt + (int64_t)lr * B * kBT;
        if (uni) {
            // 8 slots at a time: the loads issued together (clamped to the row's last slot, so
            // every address is in range), the mirrored sums of the 8 slots reduced over the
            // lanes by one butterfly that leaves slot s0 + q summed in lane 8 q
            for (int s0 = 0; s0 < B; s0 += 8) {
                double a[8], c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int s = s0 + u;
                    const double av = (double)v[(s < B ? s : B - 1) * kBT];
                    a[u] = s < B && s >= slo && s < shi ? av : 0.0;
                    c[u] = j < l ? a[u] * yj : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (a[u] != 0.0) {
                        const int s = s0 + u;
                        if (staged) atomicAdd(&s_dir[ib + s - ibase][lane], a[u] * yl);
                        else atomicAdd(x + (int64_t)(ib + s) * M + j, a[u] * yl);
                    }
                const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
                double h[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) h[u] = (b5 ? c[u + 4] : c[u]) + __shfl_xor(b5 ? c[u] : c[u + 4], 32, 64);
                double q[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) q[u] = (b4 ? h[u + 2] : h[u]) + __shfl_xor(b4 ? h[u] : h[u + 2], 16, 64);
                double w = (b3 ? q[1] : q[0]) + __shfl_xor(b3 ? q[0] : q[1], 8, 64);
                w += __shfl_xor(w, 1, 64);
                w += __shfl_xor(w, 2, 64);
                w += __shfl_xor(w, 4, 64);
                const int s = s0 + (lane >> 3);
                if ((lane & 7) == 0 && s < B && s >= slo0 && s < shi0 && w != 0.0) {
                    if (staged) atomicAdd(&s_mir[ib0 + s - ibase][lr], w);
                    else atomicAdd(x + (int64_t)(ib0 + s) * M + l, w);
                }
            }
            continue;
        }
        for (int s = 0; s < B; ++s) {
            const bool in = s >= slo && s < shi;
            const double a = in ? (double)v[s * kBT] : 0.0;
            if (a != 0.0) {
                if (staged) atomicAdd(&s_dir[ib + s - ibase][lane], a * yl);
                else atomicAdd(x + (int64_t)(ib + s) * M + j, a * yl);
            }
            const double c = (in && j < l) ? a * yj : 0.0;
            if (c != 0.0) {
                if (staged) atomicAdd(&s_mir[ib + s - ibase][lr], c);
                else atomicAdd(x + (int64_t)(ib + s) * M + l, c);
            }
        }
    }
    if (!staged) return;
    __syncthreads();
    for (int e = threadIdx.x; e < span * kBT; e += 256) {
        const int r = e / kBT, q = e % kBT;
        const double d = s_dir[r][q], mm = s_mir[r][q];
        if (d != 0.0 && tj * kBT + q < M) atomicAdd(x + (int64_t)(ibase + r) * M + tj * kBT + q, d);
        if (mm != 0.0 && tl * kBT + q < M) atomicAdd(x + (int64_t)(ibase + r) * M + tl * kBT + q, mm);
    }
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_lp_round(int64_t P, const float* p, uint16_t* q, hipStream_t s)
{
    hipLaunchKernelGGL(k_lp_round, dim3(blocks_for(P, 256)), dim3(256), 0, s, P, p, q);
}

// sc[0] = s = sqrt(vv / n), sc[1] = 1/s (0 for s = 0: then the network's output is exactly 0)
__global__ void k_lp_scale(const double* __restrict__ vv, int64_t n, double* __restrict__ sc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double s = sqrt(fmax(vv[0], 0.0) / (double)n);
        sc[0] = s;
        sc[1] = s > 0.0 ? 1.0 / s : 0.0;
    }
}

void launch_lp_scale(const double* vv, int64_t n, double* sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_lp_scale, dim3(1), dim3(64), 0, st, vv, n, sc);
}

void launch_lp_forward(LpGraph g, int layers, const float* params, const uint16_t* wq, const double* v,
                       const double* sc, float* H, int64_t hstride, float* U, double* z, hipStream_t st)
{
    const int64_t n = (int64_t)g.N * g.M;
    hipLaunchKernelGGL(k_lp_input, dim3(blocks_for(n * kH, 256)), dim3(256), 0, st, n, g, v, sc,
                       wq + lp_off_win(), params + lp_off_bin(), H);
    for (int l = 0; l < layers; ++l) {
        const float* hin = H + (hstride ? l * hstride : (l & 1) * n * kH);
        float* hout = H + (hstride ? (l + 1) * hstride : ((l + 1) & 1) * n * kH);
        hipLaunchKernelGGL(k_lp_layer, dim3(blocks_for(n, kTile)), dim3(256), 0, st, n, g, hin,
                           wq + lp_off_w(l), params + lp_off_b(l), hout, U ? U + l * n * kH : nullptr);
    }
    const float* hl = H + (hstride ? layers * hstride : (layers & 1) * n * kH);
    hipLaunchKernelGGL(k_lp_output, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, hl, wq + lp_off_wout(layers),
                       sc, z);
}

int lp_partial_blocks(int64_t n) { return (int)blocks_for(n, kChunk); }

void launch_lp_backward(LpGraph g, int layers, const uint16_t* wq, const double* v, const double* sc,
                        const float* H, const float* U, const double* dz, float* dH2, float* DU, float* dX,
                        float* partial, float* grad, hipStream_t st)
{
    const int64_t n = (int64_t)g.N * g.M;
    const int nb = lp_partial_blocks(n);
    float* dh = dH2;
    float* dh_next = dH2 + n * kH;
    hipLaunchKernelGGL(k_lp_output_bwd, dim3(nb), dim3(256), 0, st, n, H + layers * n * kH,
                       wq + lp_off_wout(layers), sc, dz, dh, partial);
    hipLaunchKernelGGL(k_lp_reduce, dim3(1), dim3(256), 0, st, partial, nb, kH, grad + lp_off_wout(layers));
    for (int l = layers - 1; l >= 0; --l) {
        const float* hin = H + l * n * kH;
        hipLaunchKernelGGL(k_lp_layer_bwd_dx, dim3(blocks_for(n, kTile)), dim3(256), 0, st, n, U + l * n * kH, dh,
                           wq + lp_off_w(l), DU, dX);
        hipLaunchKernelGGL(k_lp_layer_bwd_dw, dim3(nb), dim3(256), 0, st, n, g, hin, DU, partial);
        const int width = kH * 4 * kH + kH;
        hipLaunchKernelGGL(k_lp_reduce, dim3(blocks_for(width, 256)), dim3(256), 0, st, partial, nb, width,
                           grad + lp_off_w(l));
        hipLaunchKernelGGL(k_lp_layer_bwd_gather, dim3(blocks_for(n * kH, 256)), dim3(256), 0, st, n, g, dh, dX,
                           dh_next);
        float* tmp = dh;
        dh = dh_next;
        dh_next = tmp;
    }
    hipLaunchKernelGGL(k_lp_input_bwd, dim3(nb), dim3(256), 0, st, n, g, v, sc, dh, partial);
    hipLaunchKernelGGL(k_lp_reduce, dim3(1), dim3(256), 0, st, partial, nb, 4 * kH, grad + lp_off_win());
}

void launch_lp_adam(int64_t P, float* p, const float* grad, float* m, float* v2, float lr, int64_t step,
                    float gscale, uint16_t* q, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_lp_adam, dim3(blocks_for(P, 256)), dim3(256), 0, s, P, p, grad, m, v2, lr, b1, b2, 1e-8f,
                       bc1, bc2, gscale, q);
}

void launch_lp_randn(int64_t n, uint64_t seed, uint64_t stream, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lp_randn, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, seed, stream, out);
}

void launch_lp_smooth(LpGraph g, const double* x, double* y, hipStream_t s)
{
    const int64_t n = (int64_t)g.N * g.M;
    hipLaunchKernelGGL(k_lp_smooth, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, g, x, y);
}

void launch_matvec_transpose(BandView band, const double* val, const float* valf, const double* y, double* x,
                             hipStream_t s)
{
    launch_fill(x, 0.0, (int64_t)band.N * band.M, s);
    dim3 grid((unsigned)band.nt, (unsigned)band.N);
    if (valf)
        hipLaunchKernelGGL(k_matvec_tri_t<float>, grid, dim3(256), 0, s, band, valf, y, x);
    else
        hipLaunchKernelGGL(k_matvec_tri_t<double>, grid, dim3(256), 0, s, band, val, y, x);
}

}  // namespace tdbem
