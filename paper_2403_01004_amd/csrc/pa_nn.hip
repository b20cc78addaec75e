// pa_nn.hip -- the learned preconditioner's network on gfx950.
//
// N(c): three 3x3x3 convolutions over the cell grid, 8 -> 16 (+bias, ReLU)
// -> 16 (+bias, ReLU) -> 1, zero padding in r and theta, periodic in phi.
// Activations are stored point-major [cell][channel] in BF16; weights are
// FP32 masters converted to BF16 operand tables; every dense contraction
// (forward, input gradient, weight gradient) runs on the matrix cores as an
// implicit GEMM with v_mfma_f32_16x16x32_bf16 (FP32 accumulation):
//   forward / input gradient   D[co][point] = W[co][k] . X[k][point],
//                              k = tap * CIN + ci  (im2col gathered on the fly)
//   weight gradient            D[co][k] = G[co][point] . X[point][k],
//                              summed over points (bias = an all-ones column).
// MFMA operand layout (16x16x32): lane l holds A[l%16][8(l/16)+q],
// B[8(l/16)+q][l%16] (q = 0..7) and D[4(l/16)+r][l%16] (r = 0..3).
#include "pa_internal.h"

namespace pa {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Grids are batches of nb elements of nr x nt x np cells stacked along r
// (level I = b*nr + i).  Neighbour of cell (I, j, k) at tap t = (di+1)*9 +
// (dj+1)*3 + (dk+1); -1 outside the element's radial / colatitude range
// (zero padding); phi periodic when `per`, else zero padded.
__device__ __forceinline__ long nb_index(int I, int i, int j, int k, int t, int nr, int nt, int np,
                                         int per)
{
    const int di = t / 9 - 1, dj = (t / 3) % 3 - 1, dk = t % 3 - 1;
    const int ii = i + di, jj = j + dj;
    if (ii < 0 || ii >= nr || jj < 0 || jj >= nt) return -1;
    int kk = k + dk;
    if (kk < 0 || kk >= np) {
        if (!per) return -1;
        kk = kk < 0 ? kk + np : kk - np;
    }
    return ((long)(I + di) * nt + jj) * np + kk;
}

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int q = 0; q < 8; ++q) z[q] = (__bf16)0.0f;
    return z;
}

// ---------------------------------------------------------------- weights

// FP32 master -> BF16 operand tables (row = output channel of the GEMM):
//   f1 [16][224]: W1[co][ci][t] at k = t*8 + ci
//   f2 [16][448]: W2[co][ci][t] at k = t*16 + ci
//   f3 [16][448]: row 0 = W3[0][ci][t] at k = t*16 + ci, rows 1..15 zero
//   d3 [16][32] : input gradient of layer 3, row ci, k = t: W3[0][ci][26-t]
//   d2 [16][448]: input gradient of layer 2, row ci, k = t*16 + co: W2[co][ci][26-t]
__global__ void k_prep_weights(const float* th, __bf16* f1, __bf16* f2, __bf16* f3, __bf16* d3,
                               __bf16* d2)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const float* W1 = th + NN_OFF_W1;
    const float* W2 = th + NN_OFF_W2;
    const float* W3 = th + NN_OFF_W3;
    if (x < 16 * 224) {
        const int row = x / 224, k = x % 224, t = k / 8, ci = k % 8;
        f1[x] = (__bf16)(t < 27 ? W1[(row * 8 + ci) * 27 + t] : 0.0f);
    }
    if (x < 16 * 448) {
        const int row = x / 448, k = x % 448, t = k / 16, c = k % 16;
        f2[x] = (__bf16)(t < 27 ? W2[(row * 16 + c) * 27 + t] : 0.0f);
        f3[x] = (__bf16)(t < 27 && row == 0 ? W3[c * 27 + t] : 0.0f);
        d2[x] = (__bf16)(t < 27 ? W2[(c * 16 + row) * 27 + (26 - t)] : 0.0f);
    }
    if (x < 16 * 32) {
        const int row = x / 32, t = x % 32;
        d3[x] = (__bf16)(t < 27 ? W3[row * 27 + (26 - t)] : 0.0f);
    }
}

void launch_nn_prep_weights(const float* theta, NNWeights& w, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep_weights, dim3((16 * 448 + 255) / 256), dim3(256), 0, s, theta, w.f1,
                       w.f2, w.f3, w.d3, w.d2);
}

// ---------------------------------------------------------------- convolution

// Shape of one network launch: nb elements of nr x nt x np cells.
struct NNGrid {
    int nlev;  // nb * nr
    int nr, nt, np, per;
};

// Tiled convolution.  A workgroup owns a 16 (phi) x 16 (theta) tile of one
// element and marches a chunk of kConvRch radial levels.  The input planes
// of the tile with a one-cell halo ring (18 x 18 cells, all channels) sit in
// a ring of four LDS slots: output level i reads the planes of i - 1, i and
// i + 1, while the plane of i + 2 is loaded into registers; so each input
// value is read from memory once per chunk and the 27-point gathers of the
// implicit GEMM are LDS reads.  Planes and cells outside the element's
// radial or colatitude range (and outside phi when not periodic) hold zeros.
// Wave w computes rows 4w .. 4w + 3 of the tile, each row as 16 points x 16
// output channels on the matrix cores, with K = 27 * CIN (padded to a
// multiple of 32) taken in the same order as the operand tables: k = tap *
// CIN + ci, tap = (di + 1) * 9 + (dj + 1) * 3 + (dk + 1).
constexpr int kConvT = 16;                     // tile edge (cells)
constexpr int kConvH = kConvT + 2;             // with the halo ring
constexpr int kConvPlane = kConvH * kConvH;    // 324 cells
constexpr int kConvRch = 16;                   // levels per workgroup

template <int CIN>
struct ConvChunk {
    // one load slot: 8 channels (16 B) of a cell, or one value when CIN == 1
    static constexpr int per_cell = CIN >= 8 ? CIN / 8 : 1;
    static constexpr int count = kConvPlane * per_cell;
    static constexpr int per_thread = (count + 255) / 256;
};

template <int CIN>
__device__ __forceinline__ void conv_load_plane(const NNGrid& gd, const __bf16* x, long ebase,
                                                int lv, int j0, int k0, uint4 (&reg)[ConvChunk<CIN>::per_thread])
{
    using C = ConvChunk<CIN>;
    const bool lv_ok = lv >= 0 && lv < gd.nr;
#pragma unroll
    for (int q = 0; q < C::per_thread; ++q) {
        const int c = threadIdx.x + 256 * q;
        uint4 v = {0u, 0u, 0u, 0u};
        if (c < C::count && lv_ok) {
            const int cell = c / C::per_cell, part = c % C::per_cell;
            const int j = j0 - 1 + cell / kConvH;
            int k = k0 - 1 + cell % kConvH;
            // only k = -1 and k = np are ever a real cell's neighbour
            bool ok = j >= 0 && j < gd.nt && k <= gd.np;
            if (k < 0 || k == gd.np) {
                if (gd.per) k = k < 0 ? gd.np - 1 : 0;
                else ok = false;
            }
            if (ok) {
                const long p = ((ebase + lv) * gd.nt + j) * gd.np + k;
                if constexpr (CIN >= 8) v = *(const uint4*)(x + p * CIN + 8 * part);
                else v.x = (unsigned)*(const unsigned short*)(x + p);
            }
        }
        reg[q] = v;
    }
}

template <int CIN>
__device__ __forceinline__ void conv_store_plane(__bf16* slot, const uint4 (&reg)[ConvChunk<CIN>::per_thread])
{
    using C = ConvChunk<CIN>;
#pragma unroll
    for (int q = 0; q < C::per_thread; ++q) {
        const int c = threadIdx.x + 256 * q;
        if (c < C::count) {
            if constexpr (CIN >= 8) *(uint4*)(slot + 8 * c) = reg[q];
            else *(unsigned short*)(slot + c) = (unsigned short)reg[q].x;
        }
    }
}

// EPI 0: + bias, ReLU -> BF16 [p][16];  EPI 1: row 0 -> FP32 [p];
// EPI 2: times (mask[p][co] > 0) -> BF16 [p][16] (input gradient through ReLU)
// The launch is skipped when *done != 0 (done may be null).
template <int CIN, int EPI>
__global__ __launch_bounds__(256) void k_conv(NNGrid gd, const int* done, const __bf16* x,
                                              const __bf16* W, const float* bias,
                                              const __bf16* mask, void* out)
{
    constexpr int KP = ((27 * CIN + 31) / 32) * 32;
    constexpr int NCH = KP / 32;
    constexpr int SLOT = kConvPlane * CIN;
    __shared__ __align__(16) __bf16 sh[4 * SLOT];
    if (done && *done) return;
    const int nr = gd.nr, nt = gd.nt, np = gd.np;
    const int ntk = (np + kConvT - 1) / kConvT, ntj = (nt + kConvT - 1) / kConvT;
    const int nrc = (nr + kConvRch - 1) / kConvRch;
    int L = blockIdx.x;
    const int tk = L % ntk;
    L /= ntk;
    const int tj = L % ntj;
    L /= ntj;
    const int rc = L % nrc, e = L / nrc;
    const int k0 = tk * kConvT, j0 = tj * kConvT;
    const int i0 = rc * kConvRch, i1 = min(nr, i0 + kConvRch);
    const long ebase = (long)e * nr;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    // this lane's A operands (weights): row n, k = 32 ch + 8 g .. + 7
    bf16x8 A[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) A[ch] = *(const bf16x8*)(W + n * KP + ch * 32 + 8 * g);
    uint4 reg[ConvChunk<CIN>::per_thread];
    conv_load_plane<CIN>(gd, x, ebase, i0 - 1, j0, k0, reg);
    conv_store_plane<CIN>(sh + ((i0 + 3) & 3) * SLOT, reg);
    conv_load_plane<CIN>(gd, x, ebase, i0, j0, k0, reg);
    conv_store_plane<CIN>(sh + ((i0 + 4) & 3) * SLOT, reg);
    conv_load_plane<CIN>(gd, x, ebase, i0 + 1, j0, k0, reg);
    for (int lv = i0; lv < i1; ++lv) {
        conv_store_plane<CIN>(sh + ((lv + 5) & 3) * SLOT, reg);
        if (lv + 2 <= i1) conv_load_plane<CIN>(gd, x, ebase, lv + 2, j0, k0, reg);
        __syncthreads();
        f32x4 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 4 * wv + q;
                bf16x8 b;
                if constexpr (CIN >= 8) {
                    constexpr int TPC = 32 / CIN;         // taps per chunk (2 or 4)
                    constexpr int LPT = 4 / TPC;          // lane groups per tap
                    const int t = ch * TPC + g / LPT;
                    if (t < 27) {
                        const int di = t / 9 - 1, dj = (t / 3) % 3 - 1, dk = t % 3 - 1;
                        const __bf16* s = sh + ((lv + 4 + di) & 3) * SLOT;
                        const int cell = (row + 1 + dj) * kConvH + (n + 1 + dk);
                        b = *(const bf16x8*)(s + cell * CIN + 8 * (g % LPT));
                    } else {
                        b = zero8();
                    }
                } else {  // CIN == 1: the lane's eight k are eight taps
#pragma unroll
                    for (int qq = 0; qq < 8; ++qq) {
                        const int t = 8 * g + qq;
                        if (t < 27) {
                            const int di = t / 9 - 1, dj = (t / 3) % 3 - 1, dk = t % 3 - 1;
                            const __bf16* s = sh + ((lv + 4 + di) & 3) * SLOT;
                            b[qq] = s[(row + 1 + dj) * kConvH + (n + 1 + dk)];
                        } else {
                            b[qq] = (__bf16)0.0f;
                        }
                    }
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ch], b, acc[q], 0, 0, 0);
            }
        }
        const int k = k0 + n;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + 4 * wv + q;
            if (j >= nt || k >= np) continue;
            const long p = ((ebase + lv) * nt + j) * np + k;
            if constexpr (EPI == 1) {
                if (g == 0) ((float*)out)[p] = acc[q][0];
            } else {
                __bf16 v4[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = 4 * g + r;
                    float v = acc[q][r];
                    if constexpr (EPI == 0) v = fmaxf(v + bias[co], 0.0f);
                    else v = ((float)mask[p * 16 + co] > 0.0f) ? v : 0.0f;
                    v4[r] = (__bf16)v;
                }
                __bf16* o = (__bf16*)out + p * 16 + 4 * g;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = v4[r];
            }
        }
    }
}

static int conv_blocks(int nb, int nr, int nt, int np)
{
    return ((np + kConvT - 1) / kConvT) * ((nt + kConvT - 1) / kConvT) *
           ((nr + kConvRch - 1) / kConvRch) * nb;
}

void launch_nn_conv(int layer, int dir, int nb, int nr, int nt, int np, int per, const int* done,
                    const __bf16* x, const NNWeights& w, const float* theta, const __bf16* mask,
                    void* out, hipStream_t s)
{
    const NNGrid gd{nb * nr, nr, nt, np, per};
    const dim3 gr(conv_blocks(nb, nr, nt, np)), bl(256);
    if (dir == 0) {  // forward
        if (layer == 1)
            hipLaunchKernelGGL((k_conv<8, 0>), gr, bl, 0, s, gd, done, x, w.f1, theta + NN_OFF_B1,
                               nullptr, out);
        else if (layer == 2)
            hipLaunchKernelGGL((k_conv<16, 0>), gr, bl, 0, s, gd, done, x, w.f2, theta + NN_OFF_B2,
                               nullptr, out);
        else
            hipLaunchKernelGGL((k_conv<16, 1>), gr, bl, 0, s, gd, done, x, w.f3, nullptr, nullptr,
                               out);
    } else {  // input gradient of `layer`, masked by the ReLU of its input
        if (layer == 3)
            hipLaunchKernelGGL((k_conv<1, 2>), gr, bl, 0, s, gd, done, x, w.d3, nullptr, mask, out);
        else
            hipLaunchKernelGGL((k_conv<16, 2>), gr, bl, 0, s, gd, done, x, w.d2, nullptr, mask, out);
    }
}

// ---------------------------------------------------------------- weight gradient

// Partial dW over a block of points: D[co][kc] = sum_p G[p][co] X[p][kc],
// kc = t*CIN + ci (< 27*CIN) or the bias column kc = 27*CIN (X = 1).
// Tiled like the convolution: a workgroup owns a 16 x 16 tile of one element
// over kWgradRch radial levels, and a level's 256 points are eight K-chunks
// of 32 (two tile rows each).  The level's G (no halo) is staged in LDS
// transposed, [co][point], so a lane's eight points of one channel are one
// 16-byte read; the input planes (with the halo, three levels) sit in a
// ring of four slots, channel-planar [ci][cell].  Points outside the mesh
// carry G = 0.  Wave w accumulates the column tiles w, w + 4, ... over all
// the workgroup's points and writes part[block][co][kc] for co < COUT,
// kc < NKC.
constexpr int kWgradRch = 32;

template <int CIN>
__device__ __forceinline__ void wgrad_store_plane(__bf16* slot, const uint4 (&reg)[ConvChunk<CIN>::per_thread])
{
    using C = ConvChunk<CIN>;
#pragma unroll
    for (int q = 0; q < C::per_thread; ++q) {
        const int c = threadIdx.x + 256 * q;
        if (c < C::count) {
            const int cell = c / C::per_cell, c0 = 8 * (c % C::per_cell);
            const __bf16* v = (const __bf16*)&reg[q];
#pragma unroll
            for (int h = 0; h < 8; ++h) slot[(c0 + h) * kConvPlane + cell] = v[h];
        }
    }
}

template <int CIN, int COUT, bool BIAS>
__global__ __launch_bounds__(256) void k_wgrad(NNGrid gd, const __bf16* X, const __bf16* G,
                                               float* part)
{
    constexpr int NKC = 27 * CIN + (BIAS ? 1 : 0);
    constexpr int NTILE = (NKC + 15) / 16;
    constexpr int TPW = (NTILE + 3) / 4;  // column tiles per wave
    constexpr int SLOT = kConvPlane * CIN;
    constexpr int GCH = COUT == 16 ? 2 : 1;  // 16-byte chunks of G per point (COUT == 1: one value)
    __shared__ __align__(16) __bf16 sx[4 * SLOT];
    __shared__ __align__(16) __bf16 sg[COUT * 256];
    const int nr = gd.nr, nt = gd.nt, np = gd.np;
    const int ntk = (np + kConvT - 1) / kConvT, ntj = (nt + kConvT - 1) / kConvT;
    const int nrc = (nr + kWgradRch - 1) / kWgradRch;
    int L = blockIdx.x;
    const int tk = L % ntk;
    L /= ntk;
    const int tj = L % ntj;
    L /= ntj;
    const int rc = L % nrc, e = L / nrc;
    const int k0 = tk * kConvT, j0 = tj * kConvT;
    const int i0 = rc * kWgradRch, i1 = min(nr, i0 + kWgradRch);
    const long ebase = (long)e * nr;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    f32x4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint4 reg[ConvChunk<CIN>::per_thread];
    conv_load_plane<CIN>(gd, X, ebase, i0 - 1, j0, k0, reg);
    wgrad_store_plane<CIN>(sx + ((i0 + 3) & 3) * SLOT, reg);
    conv_load_plane<CIN>(gd, X, ebase, i0, j0, k0, reg);
    wgrad_store_plane<CIN>(sx + ((i0 + 4) & 3) * SLOT, reg);
    conv_load_plane<CIN>(gd, X, ebase, i0 + 1, j0, k0, reg);
    for (int lv = i0; lv < i1; ++lv) {
        // G of this level's tile points: chunk c of point pt = c / GCH
        uint4 gr[GCH];
#pragma unroll
        for (int q = 0; q < GCH; ++q) {
            const int c = threadIdx.x + 256 * q, pt = c / GCH;
            const int j = j0 + pt / kConvT, k = k0 + pt % kConvT;
            uint4 v = {0u, 0u, 0u, 0u};
            if (j < nt && k < np) {
                const long p = ((ebase + lv) * nt + j) * np + k;
                if constexpr (COUT == 16) v = *(const uint4*)(G + p * 16 + 8 * (c % GCH));
                else v.x = (unsigned)*(const unsigned short*)(G + p);
            }
            gr[q] = v;
        }
        __syncthreads();  // the previous level's reads of sg are done
        wgrad_store_plane<CIN>(sx + ((lv + 5) & 3) * SLOT, reg);
#pragma unroll
        for (int q = 0; q < GCH; ++q) {
            const int c = threadIdx.x + 256 * q, pt = c / GCH;
            if constexpr (COUT == 16) {
                const int c0 = 8 * (c % GCH);
                const __bf16* v = (const __bf16*)&gr[q];
#pragma unroll
                for (int h = 0; h < 8; ++h) sg[(c0 + h) * 256 + pt] = v[h];
            } else {
                *(unsigned short*)(sg + pt) = (unsigned short)gr[q].x;
            }
        }
        if (lv + 2 <= i1) conv_load_plane<CIN>(gd, X, ebase, lv + 2, j0, k0, reg);
        __syncthreads();
#pragma unroll 1
        for (int ch = 0; ch < 8; ++ch) {
            // A = G^T: row co = n, points 32 ch + 8 g .. + 7
            const bf16x8 a = n < COUT ? *(const bf16x8*)(sg + n * 256 + 32 * ch + 8 * g) : zero8();
            const int row = 2 * ch + (g >> 1), col0 = 8 * (g & 1);
#pragma unroll
            for (int tq = 0; tq < TPW; ++tq) {
                const int tile = wv + 4 * tq;
                if (tile >= NTILE) break;
                const int kc = tile * 16 + n;
                bf16x8 b;
                if (kc < 27 * CIN) {
                    const int t = kc / CIN, ci = kc % CIN;
                    const int di = t / 9 - 1, dj = (t / 3) % 3 - 1, dk = t % 3 - 1;
                    const __bf16* s = sx + ((lv + 4 + di) & 3) * SLOT + ci * kConvPlane +
                                      (row + 1 + dj) * kConvH + (col0 + 1 + dk);
#pragma unroll
                    for (int q = 0; q < 8; ++q) b[q] = s[q];
                } else {
                    const __bf16 one = (BIAS && kc == 27 * CIN) ? (__bf16)1.0f : (__bf16)0.0f;
#pragma unroll
                    for (int q = 0; q < 8; ++q) b[q] = one;
                }
                acc[tq] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tq], 0, 0, 0);
            }
        }
    }
    float* pb = part + (size_t)blockIdx.x * COUT * NKC;
#pragma unroll
    for (int tq = 0; tq < TPW; ++tq) {
        const int tile = wv + 4 * tq;
        if (tile >= NTILE) break;
        const int kc = tile * 16 + n;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = 4 * g + r;
            if (co < COUT && kc < NKC) pb[co * NKC + kc] = acc[tq][r];
        }
    }
}

// The partials are summed in a fixed order in two passes: segment s of
// kWgradSeg consecutive blocks into row s of part2, then the rows of part2
// in order into grad[layer offsets].
constexpr int kWgradSeg = 64;       // blocks per first-pass segment

__global__ void k_wgrad_seg(const float* part, int nblk, int ncol, float* part2)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ncol) return;
    const int b0 = blockIdx.y * kWgradSeg, b1 = min(nblk, b0 + kWgradSeg);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += part[(size_t)b * ncol + x];
    part2[(size_t)blockIdx.y * ncol + x] = s;
}

__global__ void k_wgrad_reduce(const float* part, int nblk, int cout, int cin, int bias,
                               int off_w, int off_b, float* grad)
{
    const int nkc = 27 * cin + bias;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= cout * nkc) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * cout * nkc + x];
    const int co = x / nkc, kc = x % nkc;
    if (kc < 27 * cin) {
        const int t = kc / cin, ci = kc % cin;
        grad[off_w + (co * cin + ci) * 27 + t] += s;
    } else {
        grad[off_b + co] += s;
    }
}

static int wgrad_blocks(int nb, int nr, int nt, int np)
{
    return ((np + kConvT - 1) / kConvT) * ((nt + kConvT - 1) / kConvT) *
           ((nr + kWgradRch - 1) / kWgradRch) * nb;
}

int nn_wgrad_partials(int nb, int nr, int nt, int np)
{
    const int nblk = wgrad_blocks(nb, nr, nt, np);
    return nblk + (nblk + kWgradSeg - 1) / kWgradSeg;
}

void launch_nn_wgrad(int layer, int nb, int nr, int nt, int np, int per, const __bf16* X,
                     const __bf16* G, float* part, float* grad, hipStream_t s)
{
    const NNGrid gd{nb * nr, nr, nt, np, per};
    const int nblk = wgrad_blocks(nb, nr, nt, np);
    const int nseg = (nblk + kWgradSeg - 1) / kWgradSeg;
    const int cin = layer == 1 ? 8 : 16, cout = layer == 3 ? 1 : 16, bias = layer == 3 ? 0 : 1;
    const int ncol = cout * (27 * cin + bias);
    float* part2 = part + (size_t)nblk * ncol;
    if (layer == 1)
        hipLaunchKernelGGL((k_wgrad<8, 16, true>), dim3(nblk), dim3(256), 0, s, gd, X, G, part);
    else if (layer == 2)
        hipLaunchKernelGGL((k_wgrad<16, 16, true>), dim3(nblk), dim3(256), 0, s, gd, X, G, part);
    else
        hipLaunchKernelGGL((k_wgrad<16, 1, false>), dim3(nblk), dim3(256), 0, s, gd, X, G, part);
    hipLaunchKernelGGL(k_wgrad_seg, dim3((ncol + 255) / 256, nseg), dim3(256), 0, s, part, nblk,
                       ncol, part2);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((ncol + 255) / 256), dim3(256), 0, s, part2, nseg,
                       cout, cin, bias, layer == 1 ? NN_OFF_W1 : layer == 2 ? NN_OFF_W2 : NN_OFF_W3,
                       layer == 1 ? NN_OFF_B1 : layer == 2 ? NN_OFF_B2 : 0, grad);
}

// ---------------------------------------------------------------- features

// Static input channels, once per solve: x[p][1] = w V/D, x[p][2..7] =
// -dt L_{p,nb}/D for the six face neighbours (r-, r+, t-, t+, p-, p+).
__global__ void k_nn_static(Geo<double> g, double dt, const double* w, const double* D,
                            const double* cpl, __bf16* x)
{
    const unsigned N = (unsigned)g.nr * g.P;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        const unsigned i = m / g.P, pp = m - i * g.P, j = pp / g.np, k = pp - j * g.np;
        const double V = g.vr[i] * g.vt[j] * g.vp[k] * (w ? w[m] : 1.0);
        const double d = D[m];
        x[(size_t)m * 8 + 1] = (__bf16)(float)(V / d);
        for (int q = 0; q < 6; ++q) x[(size_t)m * 8 + 2 + q] = (__bf16)(float)(-dt * cpl[(size_t)q * N + m] / d);
    }
}

void launch_nn_static(const Geo<double>& g, double dt, const double* w, const double* D,
                      const double* cpl, __bf16* x, hipStream_t s)
{
    const size_t N = (size_t)g.nr * g.P;
    hipLaunchKernelGGL(k_nn_static, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, g, dt, w, D, cpl, x);
}

// Dynamic channel: x[p][0] = (r/D)/sigma (0 when sigma == 0)
__global__ void k_nn_c0(unsigned N, const double* r, const double* D, const double* sig,
                        const int* done, __bf16* x)
{
    if (done && *done) return;
    const double s = *sig;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x)
        x[(size_t)m * 8] = (__bf16)(float)(r[m] / D[m] * inv);
}

void launch_nn_c0(size_t N, const double* r, const double* D, const double* sigma, const int* done,
                  __bf16* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_nn_c0, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, r, D, sigma, done, x);
}

// ---------------------------------------------------------------- training

__global__ void k_sum_finish(const double* part, int n, double N, double* out);

// Jacobi diagonal of the BE system: D = w V + dt diag(L) (w null for 1)
__global__ void k_jacobi_D(Geo<double> g, double dt, const double* w, const double* dL, double* D)
{
    const unsigned N = (unsigned)g.nr * g.P;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        const unsigned i = m / g.P, pp = m - i * g.P, j = pp / g.np, k = pp - j * g.np;
        D[m] = g.vr[i] * g.vt[j] * g.vp[k] * (w ? w[m] : 1.0) + dt * dL[m];
    }
}

void launch_jacobi_D(const Geo<double>& g, double dt, const double* w, const double* dL, double* D,
                     hipStream_t s)
{
    const size_t N = (size_t)g.nr * g.P;
    hipLaunchKernelGGL(k_jacobi_D, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, g, dt, w, dL, D);
}

// Network input of one pair on the whole grid: x[.][0] = bf16((r/D)/sigma),
// x[.][1..7] = xs[.][1..7] (static channels), zj = r/D
__global__ void k_pair_build(unsigned N, const __bf16* xs, const double* r, const double* D,
                             const double* sig, __bf16* x, double* zj)
{
    const double s = *sig;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        const double z = r[m] / D[m];
        zj[m] = z;
        x[(size_t)m * 8] = (__bf16)(float)(z * inv);
#pragma unroll
        for (int c = 1; c < 8; ++c) x[(size_t)m * 8 + c] = xs[(size_t)m * 8 + c];
    }
}

void launch_pair_build(size_t N, const __bf16* xs, const double* r, const double* D,
                       const double* sig, __bf16* x, double* zj, hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_build, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, xs, r, D, sig, x, zj);
}

// d = zj + sigma out - e: the error of the preconditioned residual
__global__ void k_nn_resid(unsigned N, const double* zj, const float* out, const double* sig,
                           const double* e, double* d)
{
    const double s = *sig;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x)
        d[m] = zj[m] + s * (double)out[m] - e[m];
}

void launch_nn_resid(size_t N, const double* zj, const float* out, const double* sig,
                     const double* e, double* d, hipStream_t s)
{
    hipLaunchKernelGGL(k_nn_resid, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, zj, out, sig, e, d);
}

// gout = 2 sigma (M d) scale / den, the output gradient of
// scale * <d, M d> / den (M symmetric)
__global__ void k_energy_gout(unsigned N, const double* Md, const double* sig, const double* den,
                              double scale, __bf16* gout)
{
    const double f = 2.0 * (*sig) * scale / (*den);
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x)
        gout[m] = (__bf16)(float)(f * Md[m]);
}

void launch_energy_gout(size_t N, const double* Md, const double* sig, const double* den,
                        double scale, __bf16* gout, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_gout, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, Md, sig, den, scale, gout);
}

// t = sum of n partials (fixed order); *out = t when den is null, else
// *out += t * scale / *den
__global__ void k_scal_reduce(const double* part, int n, const double* den, double scale,
                              double* out)
{
    __shared__ double lds[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lds[w];
    if (den) *out += t * scale / *den;
    else *out = t;
}

void launch_scal_reduce(const double* part, int n, const double* den, double scale, double* out,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_scal_reduce, dim3(1), dim3(1024), 0, s, part, n, den, scale, out);
}

// out = a - b
__global__ void k_sub(unsigned N, const double* a, const double* b, double* out)
{
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x)
        out[m] = a[m] - b[m];
}

void launch_sub(size_t N, const double* a, const double* b, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, a, b, out);
}

// FP32 [N][8] BF16 features -> FP32 [8][N] (for parity checks)
__global__ void k_nn_unpack(unsigned N, const __bf16* x, float* f)
{
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x)
        for (int c = 0; c < 8; ++c) f[(size_t)c * N + m] = (float)x[(size_t)m * 8 + c];
}

void launch_nn_unpack(size_t N, const __bf16* x, float* f, hipStream_t s)
{
    hipLaunchKernelGGL(k_nn_unpack, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, x, f);
}

// z = r/D + sigma out (one component, no partials)
__global__ void k_nn_apply(unsigned N, const double* r, const double* D, const float* out,
                           const double* sig, double* z)
{
    const double s = *sig;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x)
        z[m] = r[m] / D[m] + s * (double)out[m];
}

void launch_nn_apply(size_t N, const double* r, const double* D, const float* out,
                     const double* sigma, double* z, hipStream_t s)
{
    hipLaunchKernelGGL(k_nn_apply, dim3((unsigned)((N + 255) / 256 > 4096 ? 4096 : (N + 255) / 256)),
                       dim3(256), 0, s, (unsigned)N, r, D, out, sigma, z);
}

// Adam (Kingma & Ba) on the FP32 masters; t counts from 1
__global__ void k_adam(int n, float* th, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, int t)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const float gg = grad[x];
    const float mm = b1 * m[x] + (1.0f - b1) * gg;
    const float vv = b2 * v[x] + (1.0f - b2) * gg * gg;
    m[x] = mm;
    v[x] = vv;
    const float mh = mm / (1.0f - powf(b1, (float)t));
    const float vh = vv / (1.0f - powf(b2, (float)t));
    th[x] -= lr * mh / (sqrtf(vh) + eps);
}

void launch_nn_adam(float* th, const float* grad, float* m, float* v, float lr, int t, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((NN_NPARAM + 255) / 256), dim3(256), 0, s, NN_NPARAM, th, grad,
                       m, v, lr, 0.9f, 0.999f, 1e-8f, t);
}

// ---------------------------------------------------------------- FCG pieces

// z = r/D + sigma out (or r/D when the network is off for this step);
// partials <z,q>, <z,r>, <r/D, q>
__global__ __launch_bounds__(256) void k_fcg_combine(unsigned N, int nc, const double* r,
                                                     const double* q, const double* D,
                                                     const float* out, const double* sig,
                                                     const int* done, double* z, double* part)
{
    __shared__ double lds[4];
    if (*done) return;
    const double s = *sig;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N * nc;
         m += gridDim.x * blockDim.x) {
        const unsigned cell = m % N;
        const double zj = r[m] / D[cell];
        const double zv = zj + s * (double)out[m];
        z[m] = zv;
        a0 += zv * q[m];
        a1 += zv * r[m];
        a2 += zj * q[m];
    }
    double vals[3] = {a0, a1, a2};
    for (int t = 0; t < 3; ++t) {
        double v = vals[t];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) part[(size_t)t * gridDim.x + blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
    }
}

int launch_fcg_combine(size_t N, int nc, const double* r, const double* q, const double* D,
                       const float* out, const double* sigma, const int* done, double* z,
                       double* part, hipStream_t s)
{
    const int nb = (int)((N * nc + 255) / 256 > 4096 ? 4096 : (N * nc + 255) / 256);
    hipLaunchKernelGGL(k_fcg_combine, dim3(nb), dim3(256), 0, s, (unsigned)N, nc, r, q, D, out,
                       sigma, done, z, part);
    return nb;
}

// partials of sum (r/D)^2 (one component)
__global__ __launch_bounds__(256) void k_nn_zz(unsigned N, const double* r, const double* D,
                                               const int* done, double* part)
{
    __shared__ double lds[4];
    if (done && *done) return;
    double acc = 0.0;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        const double z = r[m] / D[m];
        acc += z * z;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// *out = sqrt(sum(part) / N) (fixed order), or the plain sum when N == 0
__global__ void k_sum_finish(const double* part, int n, double N, double* out)
{
    __shared__ double lds[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
        *out = N > 0.0 ? sqrt(s / N) : s;
    }
}

void launch_nn_sigma(size_t N, const double* r, const double* D, const int* done, double* part,
                     double* sigma, hipStream_t s)
{
    const int nb = (int)((N + 255) / 256 > 1024 ? 1024 : (N + 255) / 256);
    hipLaunchKernelGGL(k_nn_zz, dim3(nb), dim3(256), 0, s, (unsigned)N, r, D, done, part);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(1024), 0, s, part, nb, (double)N, sigma);
}

void launch_sum_finish(const double* part, int n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(1024), 0, s, part, n, 0.0, out);
}

// FCG(1) scalars.  alpha = <p, r>/<p, q> (breakdown if <p, q> <= 0)
__global__ void k_fcg_alpha(const double* part, int n, DevState* st)
{
    __shared__ double lds[16];
    if (st->done) return;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double pq = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) pq += lds[w];
    st->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) { st->status = 5; st->done = 1; return; }
    st->alpha = st->rz / pq;   // rz holds <p, r> in the flexible variant
}

// after the update: stopping test on ||r||
__global__ void k_fcg_check(const double* part, int n, DevState* st)
{
    __shared__ double lds[16];
    if (st->done) return;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[n + i];   // <r, r> partials
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double rr = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) rr += lds[w];
    st->iters += 1;
    st->rr = rr;
    if (!isfinite(rr)) { st->status = 6; st->done = 1; return; }
    if (st->force_iters > 0) {
        if (st->iters >= st->force_iters) st->done = 1;
    } else {
        if (sqrt(rr) <= st->tol * sqrt(st->bb)) st->done = 1;
        else if (st->iters >= st->max_iter) { st->status = 4; st->done = 1; }
    }
}

// beta = -<z, q>/<p, q>; when <z, r> <= 0 the step falls back to z = r/D
// (beta = -<r/D, q>/<p, q>) and st->nonfinite counts the fallbacks
__global__ void k_fcg_beta(const double* part, int n, DevState* st, int* use_jacobi)
{
    __shared__ double lds[3][16];
    if (st->done) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        for (int t = 0; t < 3; ++t) v[t] += part[(size_t)t * n + i];
    for (int t = 0; t < 3; ++t) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[t] += __shfl_xor(v[t], o, 64);
        if ((threadIdx.x & 63) == 0) lds[t][threadIdx.x >> 6] = v[t];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < 3; ++t)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s[t] += lds[t][w];
    const double zq = s[0], zr = s[1], jq = s[2];
    if (!(zr > 0.0) || !isfinite(zq)) {
        *use_jacobi = 1;
        st->nonfinite += 1;
        st->beta = -jq / st->pq;
    } else {
        *use_jacobi = 0;
        st->beta = -zq / st->pq;
    }
}

// First direction of a solve (partials from k_fcg_combine with q = r):
// beta = 0, and the Jacobi step when <z, r> <= 0 or non-finite
__global__ void k_fcg_first(const double* part, int n, DevState* st, int* use_jacobi)
{
    __shared__ double lds[16];
    if (st->done) return;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[(size_t)n + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double zr = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) zr += lds[w];
    const bool jac = !(zr > 0.0) || !isfinite(zr);
    *use_jacobi = jac ? 1 : 0;
    if (jac) st->nonfinite += 1;
    st->beta = 0.0;
}

void launch_fcg_first(const double* part, int n, DevState* st, int* use_jacobi, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg_first, dim3(1), dim3(1024), 0, s, part, n, st, use_jacobi);
}

// p = z + beta p (z = zbuf, or r/D on a fallback step); partials <p, r>
__global__ __launch_bounds__(256) void k_fcg_dir(unsigned N, int nc, const double* z,
                                                 const double* r, const double* D,
                                                 const int* use_jacobi, const DevState* st,
                                                 double* p, double* part)
{
    __shared__ double lds[4];
    if (st->done) return;
    const double beta = st->beta;
    const bool jac = *use_jacobi != 0;
    double acc = 0.0;
    for (unsigned m = blockIdx.x * blockDim.x + threadIdx.x; m < N * nc;
         m += gridDim.x * blockDim.x) {
        const double zz = jac ? r[m] / D[m % N] : z[m];
        const double pv = zz + beta * p[m];
        p[m] = pv;
        acc += pv * r[m];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// <p, r> into st->rz
__global__ void k_fcg_pr(const double* part, int n, DevState* st)
{
    __shared__ double lds[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0 || st->done) return;
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
    st->rz = s;
}

void launch_fcg_alpha(const double* part, int n, DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg_alpha, dim3(1), dim3(1024), 0, s, part, n, st);
}
void launch_fcg_check(const double* part, int n, DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(1024), 0, s, part, n, st);
}
void launch_fcg_beta(const double* part, int n, DevState* st, int* use_jacobi, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(1024), 0, s, part, n, st, use_jacobi);
}
int launch_fcg_dir(size_t N, int nc, const double* z, const double* r, const double* D,
                   const int* use_jacobi, const DevState* st, double* p, double* part,
                   hipStream_t s)
{
    const int nb = (int)((N * nc + 255) / 256 > 4096 ? 4096 : (N * nc + 255) / 256);
    hipLaunchKernelGGL(k_fcg_dir, dim3(nb), dim3(256), 0, s, (unsigned)N, nc, z, r, D, use_jacobi,
                       st, p, part);
    return nb;
}
void launch_fcg_pr(const double* part, int n, DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg_pr, dim3(1), dim3(1024), 0, s, part, n, st);
}

}  // namespace pa
