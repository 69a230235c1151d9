// cnn.hip -- the learned RFI flagger.
//
// The paper removes interference with the MAD statistic (section 5, Eq. 3 and
// Eq. 4) and notes that better filtering leaves room for improvement; this
// flagger learns from those MAD labels.  Network, per 64 x 256 (spectra x
// channels) tile of one signal's power P, each tile its own zero-padded image:
//   x  = log(1 + P / m),  m = median over the tile's channels of the channel's
//        mean power over the tile's spectra (1 when that median is not > 0)
//   z1 = conv3x3(x; 1 -> 16),   a1 = ReLU(z1)
//   z2 = conv3x3(a1; 16 -> 16), a2 = ReLU(z2)
//   z3 = conv3x3(a2; 16 -> 1)   (logit; flag when sigmoid(z3) > threshold)
// with conv3x3 the "same"-size cross-correlation
//   y[o][r][c] = b[o] + sum_i sum_{u,v} w[o][i][u][v] a[i][r + u - 1][c + v - 1].
// Training minimises the mean binary cross-entropy against MAD labels with
// Adam (Kingma & Ba 2015).
//
// Two implementations:
//   * training path (FP32, VALU): layer-by-layer direct convolutions on a
//     batch of tiles with every activation kept for the backward pass, the
//     weight gradients reduced per block and then over blocks in FP64;
//   * inference (FP16 operands, FP32 accumulation, MFMA): one workgroup per
//     tile runs all three layers with the activations in LDS ring buffers and
//     writes only the flags (and optionally the logits).
#include <algorithm>
#include <type_traits>

#include "corr_internal.h"

namespace corr {
namespace {

constexpr int H = kFlagTileSpectra;   // 64 spectra per tile
constexpr int W = kFlagTileChannels;  // 256 channels per tile
constexpr int HW = kCnnPixels;
// parameter offsets in the flat vector
constexpr int kW1 = 0, kB1 = 144, kW2 = 160, kB2 = 2464, kW3 = 2480, kB3 = 2624;

// Training blocks: 8 rows x 64 columns of one tile, staged with a one-pixel halo.
constexpr int BR = 8, BC = 64;
constexpr int LR = BR + 2, LC = BC + 2;
static_assert((H / BR) * (W / BC) == kCnnBlocksPerTile, "block count");

__device__ inline void tile_coords(int tile, int64_t T, int C, int &s, int64_t &m0, int &k0) {
    const int ntk = C / W;
    const int64_t ntm = T / H;
    k0 = (tile % ntk) * W;
    const int64_t rest = tile / ntk;
    m0 = (rest % ntm) * H;
    s = (int)(rest / ntm);
}

// ------------------------------------------------------------------ training

// One workgroup per batch tile: the tile's reference level m (median of the
// 256 channel means), then x = log(1 + P / m) and the labels as 0/1 floats.
// A tile id outside the data is recorded in err and gives x = y = 0.
__global__ void __launch_bounds__(256) cnn_gather_kernel(const float *__restrict__ power,
                                                         const uint8_t *__restrict__ labels, int S, int64_t T,
                                                         int C, const int32_t *__restrict__ tiles, float *x,
                                                         float *y, uint32_t *err) {
    __shared__ float v[W];
    const int b = blockIdx.x, t = threadIdx.x;
    const int tile = tiles[b];
    const int64_t n_tiles = (int64_t)S * (T / H) * (C / W);
    float *xb = x + (int64_t)b * HW, *yb = y + (int64_t)b * HW;
    if (tile < 0 || tile >= n_tiles) {
        if (t == 0) atomicOr(err, 1u);
        for (int p = t; p < HW; p += 256) xb[p] = yb[p] = 0.f;
        return;
    }
    int s, k0;
    int64_t m0;
    tile_coords(tile, T, C, s, m0, k0);
    const int64_t base = ((int64_t)s * T + m0) * C + k0;
    float acc = 0.f;
    for (int r = 0; r < H; ++r) acc += power[base + (int64_t)r * C + t];
    v[t] = acc * (1.0f / H);
    __syncthreads();
    block_sort(v, W);
    const float med = 0.5f * (v[W / 2 - 1] + v[W / 2]);
    const float lv = med > 0.f ? med : 1.f;
    for (int r = 0; r < H; ++r) {
        const int64_t g = base + (int64_t)r * C + t;
        xb[r * W + t] = log1pf(power[g] / lv);
        yb[r * W + t] = labels ? (labels[g] ? 1.f : 0.f) : 0.f;
    }
}

// Direct 3x3 convolution over [B][CI][H][W] -> [B][CO][H][W], one 8 x 64 block
// per workgroup, two pixels (rows t/64 and t/64 + 4) per thread.
//   MODE 0  forward, input is the network input x
//   MODE 1  forward, input is z of the previous layer (ReLU applied on load)
//   MODE 2  data gradient: input is dz of the next layer, the weights are the
//           next layer's, flipped and transposed (dx[i] = sum_o w[o][i] * dy[o]
//           shifted), and the output is gated by z of this layer > 0.
template <int CI, int CO, int MODE>
__global__ void __launch_bounds__(256) cnn_conv_kernel(const float *__restrict__ in, const float *__restrict__ w,
                                                       const float *__restrict__ bias,
                                                       const float *__restrict__ gate, float *__restrict__ out) {
    __shared__ float sx[CI][LR][LC];
    const int blk = blockIdx.x % kCnnBlocksPerTile;
    const int64_t b = blockIdx.x / kCnnBlocksPerTile;
    const int r0 = (blk / (W / BC)) * BR, c0 = (blk % (W / BC)) * BC;
    const int t = threadIdx.x;
    const float *src = in + b * CI * HW;
    for (int e = t; e < CI * LR * LC; e += 256) {
        const int i = e / (LR * LC), rem = e % (LR * LC);
        const int rr = rem / LC, cc = rem % LC;
        const int r = r0 + rr - 1, c = c0 + cc - 1;
        float v = 0.f;
        if (r >= 0 && r < H && c >= 0 && c < W) {
            v = src[(int64_t)i * HW + r * W + c];
            if (MODE == 1) v = fmaxf(v, 0.f);
        }
        sx[i][rr][cc] = v;
    }
    __syncthreads();
    const int c = t % BC, ra = t / BC;
    float acc0[CO], acc1[CO];
#pragma unroll
    for (int o = 0; o < CO; ++o) acc0[o] = acc1[o] = MODE == 2 ? 0.f : bias[o];
#pragma unroll 1
    for (int i = 0; i < CI; ++i) {
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const float x0 = sx[i][ra + u][c + v], x1 = sx[i][ra + 4 + u][c + v];
#pragma unroll
                for (int o = 0; o < CO; ++o) {
                    const float wv = MODE == 2 ? w[((i * CO + o) * 3 + 2 - u) * 3 + 2 - v]
                                               : w[((o * CI + i) * 3 + u) * 3 + v];
                    acc0[o] = fmaf(wv, x0, acc0[o]);
                    acc1[o] = fmaf(wv, x1, acc1[o]);
                }
            }
    }
    const int p0 = (r0 + ra) * W + c0 + c, p1 = p0 + 4 * W;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
        const int64_t ob = (b * CO + o) * HW;
        float v0 = acc0[o], v1 = acc1[o];
        if (MODE == 2) {
            v0 = gate[ob + p0] > 0.f ? v0 : 0.f;
            v1 = gate[ob + p1] > 0.f ? v1 : 0.f;
        }
        out[ob + p0] = v0;
        out[ob + p1] = v1;
    }
}

// Weight and bias gradients of one layer over one 8 x 64 block:
//   part[blk][(o CI + i) 9 + 3u + v] = sum_p dz[o][p] a[i][p + (u - 1, v - 1)]
//   part[blk][CO CI 9 + o]          = sum_p dz[o][p]
// with a = ReLU(z_prev) (RELU_IN) or the network input.  Thread t takes the
// (o, i) pair t mod CO CI and, when there are fewer than 256 pairs, one of
// 256 / (CO CI) slices of the block's rows; the slices are summed in LDS.
template <int CI, int CO, bool RELU_IN>
__global__ void __launch_bounds__(256) cnn_wgrad_kernel(const float *__restrict__ ain, const float *__restrict__ dz,
                                                        float *__restrict__ part) {
    constexpr int NP = CI * CO, G = 256 / NP, E = NP * 9 + CO;
    static_assert(NP * G == 256 && (G == 1 || G == 16), "pair count");
    __shared__ float sa[CI][LR][LC];
    __shared__ float sd[CO][BR][BC];
    __shared__ float red[G > 1 ? 256 : 1][10];
    const int blk = blockIdx.x % kCnnBlocksPerTile;
    const int64_t b = blockIdx.x / kCnnBlocksPerTile;
    const int r0 = (blk / (W / BC)) * BR, c0 = (blk % (W / BC)) * BC;
    const int t = threadIdx.x;
    for (int e = t; e < CI * LR * LC; e += 256) {
        const int i = e / (LR * LC), rem = e % (LR * LC);
        const int rr = rem / LC, cc = rem % LC;
        const int r = r0 + rr - 1, c = c0 + cc - 1;
        float v = 0.f;
        if (r >= 0 && r < H && c >= 0 && c < W) {
            v = ain[(b * CI + i) * HW + r * W + c];
            if (RELU_IN) v = fmaxf(v, 0.f);
        }
        sa[i][rr][cc] = v;
    }
    for (int e = t; e < CO * BR * BC; e += 256) {
        const int o = e / (BR * BC), rem = e % (BR * BC);
        sd[o][rem / BC][rem % BC] = dz[(b * CO + o) * HW + (r0 + rem / BC) * W + c0 + rem % BC];
    }
    __syncthreads();
    const int q = t % NP, g = t / NP;
    const int o = q / CI, i = q % CI;
    // rows and columns of this thread's slice
    const int rb = G == 1 ? 0 : g / 2, re = G == 1 ? BR : g / 2 + 1;
    const int cb = G == 1 ? 0 : (g % 2) * (BC / 2), ce = G == 1 ? BC : cb + BC / 2;
    float acc[9], bacc = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.f;
    for (int rr = rb; rr < re; ++rr) {
        float w0[3], w1[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            w0[u] = sa[i][rr + u][cb];
            w1[u] = sa[i][rr + u][cb + 1];
        }
        for (int cc = cb; cc < ce; ++cc) {
            const float d = sd[o][rr][cc];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const float w2 = sa[i][rr + u][cc + 2];
                acc[3 * u + 0] = fmaf(d, w0[u], acc[3 * u + 0]);
                acc[3 * u + 1] = fmaf(d, w1[u], acc[3 * u + 1]);
                acc[3 * u + 2] = fmaf(d, w2, acc[3 * u + 2]);
                w0[u] = w1[u];
                w1[u] = w2;
            }
            bacc += d;
        }
    }
    float *pb = part + (int64_t)blockIdx.x * E;
    if constexpr (G > 1) {
#pragma unroll
        for (int k = 0; k < 9; ++k) red[t][k] = acc[k];
        red[t][9] = bacc;
        __syncthreads();
        if (t < NP) {
            for (int k = 0; k < 10; ++k) {
                float sum = 0.f;
                for (int gg = 0; gg < G; ++gg) sum += red[gg * NP + t][k];
                if (k < 9)
                    pb[(o * CI + i) * 9 + k] = sum;
                else if (i == 0)
                    pb[NP * 9 + o] = sum;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) pb[(o * CI + i) * 9 + k] = acc[k];
        if (i == 0) pb[NP * 9 + o] = bacc;
    }
}

// grad[e] = sum over blocks of part[blk][e], in FP64, blocks in order.
__global__ void cnn_reduce_kernel(const float *__restrict__ part, int nparts, int E, float *grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += part[(int64_t)k * E + e];
    grad[e] = (float)s;
}

// Binary cross-entropy with logits: loss terms max(z, 0) - z y + log(1 + e^-|z|)
// summed per block (FP64), dz = (sigmoid(z) - y) / n.
__global__ void __launch_bounds__(256) cnn_bce_kernel(const float *__restrict__ z, const float *__restrict__ y,
                                                      int64_t n, float *dz, double *lpart) {
    __shared__ double red[256];
    const float inv_n = (float)(1.0 / (double)n);
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const float zz = z[p], yy = y[p];
        acc += (double)(fmaxf(zz, 0.f) - zz * yy + log1pf(expf(-fabsf(zz))));
        dz[p] = (1.f / (1.f + expf(-zz)) - yy) * inv_n;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void cnn_loss_final_kernel(const double *__restrict__ lpart, int nb, int64_t n, float *loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += lpart[k];
    *loss = (float)(s / (double)n);
}

// Adam: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m c1) / (sqrt(v c2) + eps), c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t).
__global__ void cnn_adam_kernel(float *p, float *m, float *v, const float *__restrict__ g, int n, float lr,
                                float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ----------------------------------------------------------------- inference

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef short short2v __attribute__((ext_vector_type(2)));
typedef float float16v __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int XCOLS = W + 4;  // input columns: zero column on the left, three on the right
constexpr int PC = W + 2;     // activation row pitch: one zero column at each edge
constexpr int RX = 8;         // rows kept of the input, of the layer-1 output and of the tap sums
constexpr int XPITCH = 10;    // halves per input column: RX rows + 2 pad (odd dword stride)
constexpr int IWG = 512;      // 8 waves, one 32-column strip each

// Accumulator layout of a 32 x 32 MFMA: register j of lane l holds row
// 8 (j / 4) + 4 (l / 32) + j mod 4, column l mod 32.
__device__ inline int acc_row(int j, int half) { return 8 * (j / 4) + 4 * half + (j & 3); }

// Two floats -> two FP16 (round to nearest even) with negatives set to +0:
// ReLU commutes with the monotone conversion, and on FP16 bit patterns the
// signed 16-bit max against 0 clears exactly the negative values.
__device__ inline uint32_t relu_h2(float a, float b) {
    const half2v h = __builtin_convertvector((float2v){a, b}, half2v);
    const short2v m = __builtin_elementwise_max(__builtin_bit_cast(short2v, h), (short2v){0, 0});
    return __builtin_bit_cast(uint32_t, m);
}

// Byte offset of the 16-byte half `h` (channels 8h .. 8h + 7) of pixel column
// pcol in a layer-1 output row: the halves swap places by bit 2 xor bit 3 of
// the column, so the 16-byte reads of 8 (or 16) consecutive lanes cover all 32
// (or 64) LDS banks once.
__device__ inline int a1_off(int pcol, int h) { return 32 * pcol + 16 * (h ^ (((pcol >> 2) ^ (pcol >> 3)) & 1)); }

// One workgroup per compute unit, looping over tiles.  Wave w owns columns
// 32 w .. 32 w + 31 and walks the tile two rows at a time in a software
// pipeline with one barrier per step j:
//   x rows 2j + 5, 2j + 6 = log(1 + P / m) (FP16) into the input ring,
//   layer 1 for rows 2j + 2, 2j + 3,
//   layer 2 and the layer-3 tap sums for rows 2j - 2, 2j - 1,
//   the logits of rows 2j - 6, 2j - 5,
// each stage reading only what earlier steps wrote, from rings of 8 rows.
// Layer 2 of a row pair reads layer-1 rows 2j - 3 .. 2j; the first two were
// read by the previous step and stay in registers.  Layer-1 rows -1 and 64
// are zero rows in the ring.  Steps run four at a time (the ring period), so
// every ring slot is a constant.  While a tile is processed, the column sums
// of the next tile and the input rows its first step needs are fetched.
// MFMA roles (32 x 32 x 16, FP16 in, FP32 out):
//   layer 1: rows = (row slot, out channel) for two rows; K = 4 input rows x 4
//            column offsets, lane half h taking input rows 2h and 2h + 1,
//            slot j = (row 2h + j mod 2, offset j / 2): with the input stored
//            column-major each slot pair is one aligned dword (offset 3 has
//            zero weight; the bias rides on slot 7 of half 0, set to 1);
//   layer 2: rows = (row slot, out channel); one product per (input row,
//            column offset), K = 16 channels, the weights of the taps a row
//            slot does not use set to zero;
//   layer 3: U[tap][q] = sum_i w3[i][tap] a2[i][q] with rows = the 9 taps, fed
//            directly from the layer-2 accumulator (its 8 channels per lane
//            are exactly one lane's K slots), then z3[p] = b3 + sum of U over
//            the 9 shifted neighbours of p.
template <typename PT>
__global__ void __launch_bounds__(IWG) cnn_infer_kernel(const float *__restrict__ params,
                                                        const PT *__restrict__ power, int64_t T, int C,
                                                        int n_tiles, float thr_logit, float guard_m,
                                                        uint8_t *__restrict__ flags,
                                                        float *__restrict__ logits) {
    __shared__ __align__(16) _Float16 xs[XCOLS][XPITCH];  // column-major input ring (slot = (row + 1) mod 8)
    __shared__ __align__(16) _Float16 a1s[RX][PC][16];   // layer-1 ring (slot = row mod 8)
    __shared__ float us[RX][PC][9];                      // tap-sum ring (slot = row mod 8)
    __shared__ float colv[2][W];                         // column sums of even / odd rows
    __shared__ float srt[IWG / 64][W];                   // each wave's sorted channel means (guard)

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int half = lane >> 5, col = lane & 31;
    const int xc = t & (W - 1), xh = t >> 8;  // input staging: column xc, rows of parity xh

    // ---- zero border columns, written once (never overwritten below)
    for (int e = t; e < 4 * XPITCH; e += IWG) xs[(e / XPITCH) == 0 ? 0 : W + (e / XPITCH)][e % XPITCH] = (_Float16)0.f;
    for (int e = t; e < RX * 2 * 16; e += IWG) {
        const int rr = e / 32, side = (e / 16) & 1, ch = e & 15;
        a1s[rr][side ? PC - 1 : 0][ch] = (_Float16)0.f;
    }
    for (int e = t; e < RX * 2 * 9; e += IWG) {
        const int rr = e / 18, side = (e / 9) & 1, k = e % 9;
        us[rr][side ? PC - 1 : 0][k] = 0.f;
    }

    // ---- weights as MFMA A operands (lane: row = lane mod 32, K slots 8 half + j)
    const int arow = lane & 31, aslot = arow >> 4, ao = arow & 15;
    half8 A1, A3, A2[4][3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int rho = 2 * half + (j & 1), dv = j >> 1, u = rho - aslot;
        float w = (dv < 3 && u >= 0 && u <= 2) ? params[kW1 + ao * 9 + u * 3 + dv] : 0.f;
        if (half == 0 && j == 7) w = params[kB1 + ao];  // constant-1 slot: the bias
        A1[j] = (_Float16)w;
        const int ch = 8 * (j / 4) + 4 * half + (j & 3);
        A3[j] = (_Float16)(arow < 9 ? params[kW3 + ch * 9 + arow] : 0.f);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int dv = 0; dv < 3; ++dv)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int cin = 8 * half + j, u = p - aslot;
                A2[p][dv][j] = (_Float16)((u >= 0 && u <= 2) ? params[kW2 + ((ao * 16 + cin) * 3 + u) * 3 + dv] : 0.f);
            }
    float16v bias2;
#pragma unroll
    for (int j = 0; j < 16; ++j) bias2[j] = params[kB2 + (acc_row(j, half) & 15)];
    const float b3 = params[kB3];
    const float16v zero16 = {};
    const half8 zero8 = {};

    const int c0 = wv * 32;
    const int pc = c0 + col + 1;  // padded column of this lane's pixel
    const uint32_t *xl = reinterpret_cast<const uint32_t *>(&xs[c0 + col][0]);
    const uint32_t bias_and = half ? 0xFFFFFFFFu : 0x0000FFFFu;  // half 0: slot 7 := 1.0
    const uint32_t bias_or = half ? 0u : 0x3C000000u;
    char *a1base = reinterpret_cast<char *>(&a1s[0][0][0]);
    const int a1w0 = a1_off(pc, 0) + 8 * half, a1w1 = a1_off(pc, 1) + 8 * half;
    int a1rd[3];
#pragma unroll
    for (int dv = 0; dv < 3; ++dv) a1rd[dv] = a1_off(pc - 1 + dv, half);
    float *uw = &us[0][pc][0];
    const float *ur = &us[0][pc - 1][0];
    constexpr int AROW = PC * 16 * 2, UROW = PC * 9;  // bytes, floats

    auto tile_base = [&](int tl) {
        int s, k0;
        int64_t m0;
        tile_coords(tl, T, C, s, m0, k0);
        return ((int64_t)s * T + m0) * C + k0;
    };
    // First tile: column sums of rows xh, xh + 2, ... and the input rows -1 + xh,
    // 1 + xh, 3 + xh of its first steps.  Later tiles get these during the previous one.
    // Offsets inside a tile (row r, column c: r C + c < 2^24) are 32-bit;
    // tile bases are uniform 64-bit pointers.
    auto roff = [&](int r, int c) { return __umul24((uint32_t)r, (uint32_t)C) + (uint32_t)c; };
    int tile = blockIdx.x;
    // p0, p1: input rows -1 + xh, 1 + xh of a tile; p2 .. p5: rows 3 + xh ..
    // 9 + xh, the first four slots of the input ring
    float csum = 0.f, p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f, p5 = 0.f;
    if (tile < n_tiles) {
        const PT *tb = power + tile_base(tile);
#pragma unroll 8
        for (int q = 0; q < 32; ++q) csum += tb[roff(2 * q + xh, xc)];
        p0 = xh ? tb[xc] : 0.f;
        p1 = tb[roff(1 + xh, xc)];
        p2 = tb[roff(3 + xh, xc)];
        p3 = tb[roff(5 + xh, xc)];
        p4 = tb[roff(7 + xh, xc)];
        p5 = tb[roff(9 + xh, xc)];
    }
    for (; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile_base(tile);
        const PT *tb = power + base;
        const bool has_next = tile + (int)gridDim.x < n_tiles;
        const PT *tn = has_next ? power + tile_base(tile + gridDim.x) : tb;
        uint8_t *fb = flags + base;
        float *lb = logits ? logits + base : nullptr;

        // ---- reference level: median over the 256 channels of each channel's mean power
        colv[xh][xc] = csum;
        for (int e = t; e < PC * 2; e += IWG)  // layer-1 row -1 (slot 7): zero
            reinterpret_cast<uint4 *>(a1base + (RX - 1) * AROW)[e] = make_uint4(0u, 0u, 0u, 0u);
        __syncthreads();
        float cv[4], cm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) cm[q] = cv[q] = (colv[0][4 * lane + q] + colv[1][4 * lane + q]) * (1.0f / H);
        const float med = wave_median256(cv, lane);  // sorts cv
        const float inv = 1.0f / (med > 0.f ? med : 1.f);
        // column guard: the channel means are the MAD column statistic (section 5, Eq. 3
        // and 4); a column whose mean is an outlier is flagged whole.  gcol is the guard
        // bit of this lane's output column c0 + col (lane (c0 + col) / 4 holds its mean).
        uint32_t gcol = 0u;
        if (guard_m > 0.f) {
            float d[4];
            uint32_t bits = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) d[q] = fabsf(cm[q] - med);
            const float mad = wave_mad256_sorted(cv, med, lane, srt[wv]);
            const float thr = guard_m * mad / 0.6745f;
#pragma unroll
            for (int q = 0; q < 4; ++q) bits |= (d[q] > thr ? 1u : 0u) << q;
            const int oc = c0 + col;
            gcol = ((uint32_t)__shfl((int)bits, oc >> 2) >> (oc & 3)) & 1u;
        }
        // x of tile row r -> input ring slot (r + 1) mod 8, zero outside the tile
        auto x_put = [&](int r, float pv) {
            const float v = (r >= 0 && r < H) ? __logf(1.0f + pv * inv) : 0.f;
            xs[xc + 1][(r + 1) & (RX - 1)] = (_Float16)v;
        };
        x_put(-1 + xh, p0);
        x_put(1 + xh, p1);
        // input ring: step j puts row 2j + 5 + xh from slot (j + 1) mod 4 and
        // loads row 2j + 13 + xh, which step j + 4 puts, into the same slot
        float xr0 = p2, xr1 = p3, xr2 = p4, xr3 = p5, cnext = 0.f;
        csum = 0.f;
        __syncthreads();

        half8 Fa[3], Fb[3];  // layer-1 operands of rows 2j - 3, 2j - 2, read by the previous step
#pragma unroll
        for (int dv = 0; dv < 3; ++dv) Fa[dv] = Fb[dv] = zero8;

        auto step = [&](const int j, auto slot_tag) {
            constexpr int SL = decltype(slot_tag)::value;  // (j + 1) mod 4
            float &xs_slot = SL == 0 ? xr0 : SL == 1 ? xr1 : SL == 2 ? xr2 : xr3;
            // (a) input row 2j + 5 + xh; row 2j + 13 + xh is fetched for step j + 4, and row
            //     2j + 2 + xh of the next tile for its column sums (added one step later).
            //     Both loads are issued at every step (rows clamped into the tile, values
            //     past its end unused), so the loads in flight are the same on every path.
            {
                const int r = 2 * j + 5 + xh;
                x_put(r, xs_slot);
                xs_slot = tb[roff(r + 8 < H ? r + 8 : H - 1, xc)];
                if (j >= 0 && j <= H / 2 - 1) csum += cnext;
                const int rc = 2 * j + 2 + xh;
                const float cn = tn[roff(rc < H ? (rc > 0 ? rc : 0) : H - 1, xc)];
                cnext = (j <= H / 2 - 2 && has_next) ? cn : 0.f;
                if (j == H / 2 && has_next) {
                    p0 = xh ? tn[xc] : 0.f;
                    p1 = tn[roff(1 + xh, xc)];
                    p2 = tn[roff(3 + xh, xc)];
                    p3 = tn[roff(5 + xh, xc)];
                    p4 = tn[roff(7 + xh, xc)];
                    p5 = tn[roff(9 + xh, xc)];
                }
            }
            // (b) layer 1 for rows R, R + 1, R = 2j + 2 (input rows R - 1 .. R + 2); row 64 is zero
            const int R = 2 * j + 2;
            if (R < H) {
                const uint32_t *xr = xl + (((R + 2 * half) & (RX - 1)) >> 1);
                u32x4 bx;
#pragma unroll
                for (int dv = 0; dv < 4; ++dv) bx[dv] = xr[dv * (XPITCH / 2)];
                bx[3] = (bx[3] & bias_and) | bias_or;
                const float16v D =
                    __builtin_amdgcn_mfma_f32_32x32x16_f16(A1, __builtin_bit_cast(half8, bx), zero16, 0, 0, 0);
#pragma unroll
                for (int sl = 0; sl < 2; ++sl) {
                    char *row = a1base + ((R + sl) & (RX - 1)) * AROW;
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const int j0 = 8 * sl + 4 * g;
                        uint2 v;
                        v.x = relu_h2(D[j0 + 0], D[j0 + 1]);
                        v.y = relu_h2(D[j0 + 2], D[j0 + 3]);
                        *reinterpret_cast<uint2 *>(row + (g ? a1w1 : a1w0)) = v;
                    }
                }
            } else if (R == H) {
                char *row = a1base + (R & (RX - 1)) * AROW;
                *reinterpret_cast<uint2 *>(row + a1w0) = make_uint2(0u, 0u);
                *reinterpret_cast<uint2 *>(row + a1w1) = make_uint2(0u, 0u);
            }
            // (c) layer 2 and the tap sums for rows r2, r2 + 1, r2 = 2j - 2 (layer-1 rows r2 - 1 .. r2 + 2)
            if (j >= 0 && j <= H / 2) {
                half8 Fc[3], Fd[3];  // layer-1 rows 2j - 1, 2j
                const char *fc = a1base + ((2 * j - 1) & (RX - 1)) * AROW;
                const char *fd = a1base + ((2 * j) & (RX - 1)) * AROW;
#pragma unroll
                for (int dv = 0; dv < 3; ++dv) {
                    Fc[dv] = *reinterpret_cast<const half8 *>(fc + a1rd[dv]);
                    Fd[dv] = *reinterpret_cast<const half8 *>(fd + a1rd[dv]);
                }
                if (j >= 1) {
                    const int r2 = 2 * j - 2;
                    float16v D = bias2;
#pragma unroll
                    for (int dv = 0; dv < 3; ++dv) D = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[0][dv], Fa[dv], D, 0, 0, 0);
#pragma unroll
                    for (int dv = 0; dv < 3; ++dv) D = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[1][dv], Fb[dv], D, 0, 0, 0);
#pragma unroll
                    for (int dv = 0; dv < 3; ++dv) D = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[2][dv], Fc[dv], D, 0, 0, 0);
#pragma unroll
                    for (int dv = 0; dv < 3; ++dv) D = __builtin_amdgcn_mfma_f32_32x32x16_f16(A2[3][dv], Fd[dv], D, 0, 0, 0);
#pragma unroll
                    for (int sl = 0; sl < 2; ++sl) {
                        u32x4 bu;
#pragma unroll
                        for (int q = 0; q < 4; ++q) bu[q] = relu_h2(D[8 * sl + 2 * q], D[8 * sl + 2 * q + 1]);
                        const float16v U =
                            __builtin_amdgcn_mfma_f32_32x32x16_f16(A3, __builtin_bit_cast(half8, bu), zero16, 0, 0, 0);
                        float *dst = uw + ((r2 + sl) & (RX - 1)) * UROW;
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[4 * half + q] = U[q];
                        if (half == 0) dst[8] = U[4];
                    }
                }
#pragma unroll
                for (int dv = 0; dv < 3; ++dv) {
                    Fa[dv] = Fc[dv];
                    Fb[dv] = Fd[dv];
                }
            }
            // (d) logits of rows 2j - 6 (lanes 0-31) and 2j - 5 (lanes 32-63)
            const int r3 = 2 * j - 6;
            if (r3 >= 0 && r3 < H) {
                const int r = r3 + half;
                float z = b3;
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const int rr = r + u - 1;
                    const float *row = ur + (rr & (RX - 1)) * UROW;
                    float zu = 0.f;
#pragma unroll
                    for (int v = 0; v < 3; ++v) zu += row[9 * v + 3 * u + v];
                    z += (rr >= 0 && rr < H) ? zu : 0.f;
                }
                const uint32_t gp = roff(r, c0 + col);
                fb[gp] = (uint8_t)((z > thr_logit ? 1u : 0u) | gcol);
                if (lb) lb[gp] = z;
            }
            __syncthreads();
        };
        // steps -1 .. 34, four at a time: 2j mod 8 is fixed within each group
        for (int i = 0; i < (H / 2 + 4) / 4; ++i) {
            const int jb = 4 * i - 1;
            step(jb, std::integral_constant<int, 0>{});
            step(jb + 1, std::integral_constant<int, 1>{});
            step(jb + 2, std::integral_constant<int, 2>{});
            step(jb + 3, std::integral_constant<int, 3>{});
        }
    }
}

}  // namespace

hipError_t launch_cnn_gather(const float *power, const uint8_t *labels, int S, int64_t T, int C,
                             const int32_t *tiles, int n, const CnnTrainBufs &b, hipStream_t st) {
    hipLaunchKernelGGL(cnn_gather_kernel, dim3(n), dim3(256), 0, st, power, labels, S, T, C, tiles, b.x, b.y, b.err);
    return hipGetLastError();
}

hipError_t launch_cnn_forward(const float *params, int n, const CnnTrainBufs &b, hipStream_t st) {
    const dim3 grid(n * kCnnBlocksPerTile), blk(256);
    hipLaunchKernelGGL((cnn_conv_kernel<1, 16, 0>), grid, blk, 0, st, b.x, params + kW1, params + kB1, nullptr, b.z1);
    hipLaunchKernelGGL((cnn_conv_kernel<16, 16, 1>), grid, blk, 0, st, b.z1, params + kW2, params + kB2, nullptr, b.z2);
    hipLaunchKernelGGL((cnn_conv_kernel<16, 1, 1>), grid, blk, 0, st, b.z2, params + kW3, params + kB3, nullptr, b.z3);
    return hipGetLastError();
}

hipError_t launch_cnn_backward(const float *params, int n, const CnnTrainBufs &b, float *grad, float *loss,
                               hipStream_t st) {
    const int64_t npx = (int64_t)n * HW;
    const int nb = (int)std::min<int64_t>(kCnnLossBlocks, (npx + 255) / 256);
    hipLaunchKernelGGL(cnn_bce_kernel, dim3(nb), dim3(256), 0, st, b.z3, b.y, npx, b.d3, b.lpart);
    hipLaunchKernelGGL(cnn_loss_final_kernel, dim3(1), dim3(64), 0, st, b.lpart, nb, npx, loss);
    const dim3 grid(n * kCnnBlocksPerTile), blk(256);
    const int nparts = n * kCnnBlocksPerTile;
    // layer 3: weights from a2 = ReLU(z2) and dz3; dz2 = (W3^T * dz3) gated by z2 > 0
    hipLaunchKernelGGL((cnn_wgrad_kernel<16, 1, true>), grid, blk, 0, st, b.z2, b.d3, b.part);
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3(1), dim3(256), 0, st, b.part, nparts, 16 * 9 + 1, grad + kW3);
    hipLaunchKernelGGL((cnn_conv_kernel<1, 16, 2>), grid, blk, 0, st, b.d3, params + kW3, nullptr, b.z2, b.d2);
    // layer 2
    hipLaunchKernelGGL((cnn_wgrad_kernel<16, 16, true>), grid, blk, 0, st, b.z1, b.d2, b.part);
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3((kCnnGradEntries + 255) / 256), dim3(256), 0, st, b.part, nparts,
                       kCnnGradEntries, grad + kW2);
    hipLaunchKernelGGL((cnn_conv_kernel<16, 16, 2>), grid, blk, 0, st, b.d2, params + kW2, nullptr, b.z1, b.d1);
    // layer 1
    hipLaunchKernelGGL((cnn_wgrad_kernel<1, 16, false>), grid, blk, 0, st, b.x, b.d1, b.part);
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3(1), dim3(256), 0, st, b.part, nparts, 16 * 9 + 16, grad + kW1);
    return hipGetLastError();
}

hipError_t launch_cnn_adam(float *params, float *m, float *v, const float *grad, float lr, float beta1,
                           float beta2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(cnn_adam_kernel, dim3((kCnnParams + 255) / 256), dim3(256), 0, st, params, m, v, grad,
                       kCnnParams, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_cnn_infer(const float *params, const void *power, bool f16, int S, int64_t T, int C,
                            float thr_logit, float guard_m, uint8_t *flags, float *logits, hipStream_t st) {
    const int n_tiles = (int)((int64_t)S * (T / H) * (C / W));
    // persistent: one workgroup per compute unit (the LDS use allows one), each
    // fetching its next tile's power while it computes the current one
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int grid = std::max(1, std::min(n_tiles, cus));
    if (f16)
        hipLaunchKernelGGL(cnn_infer_kernel<_Float16>, dim3(grid), dim3(IWG), 0, st, params,
                           static_cast<const _Float16 *>(power), T, C, n_tiles, thr_logit, guard_m, flags, logits);
    else
        hipLaunchKernelGGL(cnn_infer_kernel<float>, dim3(grid), dim3(IWG), 0, st, params,
                           static_cast<const float *>(power), T, C, n_tiles, thr_logit, guard_m, flags, logits);
    return hipGetLastError();
}

}  // namespace corr
