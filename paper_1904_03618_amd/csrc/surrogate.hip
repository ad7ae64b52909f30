// surrogate.hip -- gfx950 kernels of the learned surrogate (include/lbcg_surrogate.h):
// 3D convolutions as implicit GEMMs on the CDNA4 matrix cores
// (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation), their data and
// weight gradients, and the element-wise layers, loss and optimiser of a U-Net.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "lbcg_surrogate.h"

namespace sg {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One MFMA 16x16x32 step.  Lane l (0..63) supplies A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16] for j = 0..7, and receives
// D[4 (l / 16) + j][l % 16] for j = 0..3.
__device__ inline f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline int64_t npos(const sg_view &v) { return (int64_t)v.n * v.d * v.h * v.w; }

struct Pos { int n, z, y, x; };

__device__ inline Pos decode(const sg_view &v, int64_t p)
{
    Pos q;
    q.x = (int)(p % v.w);
    p /= v.w;
    q.y = (int)(p % v.h);
    p /= v.h;
    q.z = (int)(p % v.d);
    q.n = (int)(p / v.d);
    return q;
}

// Neighbour at offset (dz, dy, dx): flat position, or -1 where zero padding applies.
__device__ inline int64_t shifted(const sg_view &v, const Pos &q, int dz, int dy, int dx, int pmask)
{
    int z = q.z + dz, y = q.y + dy, x = q.x + dx;
    if (x < 0 || x >= v.w) {
        if (!(pmask & 1)) return -1;
        x = x < 0 ? x + v.w : x - v.w;
    }
    if (y < 0 || y >= v.h) {
        if (!(pmask & 2)) return -1;
        y = y < 0 ? y + v.h : y - v.h;
    }
    if (z < 0 || z >= v.d) {
        if (!(pmask & 4)) return -1;
        z = z < 0 ? z + v.d : z - v.d;
    }
    return (((int64_t)q.n * v.d + z) * v.h + y) * v.w + x;
}

__device__ inline void tap_offset(int tap, int k, int &dz, int &dy, int &dx)
{
    if (k == 1) {
        dz = dy = dx = 0;
        return;
    }
    dz = tap / 9 - 1;
    dy = (tap / 3) % 3 - 1;
    dx = tap % 3 - 1;
}

// ------------------------------------------------------------- forward
// Workgroup: 4 wavefronts; each wave owns a register tile of NO blocks of 16
// output channels x FP blocks of 16 positions (64 consecutive positions), so
// one weight fragment feeds FP MFMAs and one input fragment feeds NO of them.
// blockIdx.y selects the 16 NO output channels.  The K loop walks taps x
// input channels in groups of 8 (one 16-byte load per lane and operand).
constexpr int FP = 4;

template <int NO>
__global__ __launch_bounds__(256) void k_conv_fwd(sg_view x, const bf16 *__restrict__ W,
                                                  const float *__restrict__ bias, int k, int pmask, int relu,
                                                  sg_view y, sg_view y32, int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t P = npos(x);
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * FP);
    const int co0 = blockIdx.y * 16 * NO;
    const int ci = x.c, g8 = ci >> 3, taps = k * k * k;
    const int K8 = taps * g8, K = taps * ci;
    Pos q[FP];
    bool pv[FP];
    #pragma unroll
    for (int i = 0; i < FP; ++i) {
        const int64_t pb = p0 + 16 * i + col;
        pv[i] = pb < P;
        q[i] = decode(x, pv[i] ? pb : 0);
    }
    const bf16 *xp = reinterpret_cast<const bf16 *>(x.p) + x.coff;
    const bf16 *wrow = W + (int64_t)(co0 + col) * K;
    f32x4 acc[NO][FP];
    #pragma unroll
    for (int o = 0; o < NO; ++o)
        #pragma unroll
        for (int i = 0; i < FP; ++i) acc[o][i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    int last_tap = -1;
    int64_t src[FP];
    #pragma unroll
    for (int i = 0; i < FP; ++i) src[i] = -1;
    for (int kb = 0; kb < (K8 + 3) >> 2; ++kb) {
        const int g = (kb << 2) + grp;
        bf16x8 a[NO], b[FP];
        #pragma unroll
        for (int o = 0; o < NO; ++o) a[o] = zero;
        #pragma unroll
        for (int i = 0; i < FP; ++i) b[i] = zero;
        if (g < K8) {
            const int tap = g / g8, c8 = g - tap * g8;
            #pragma unroll
            for (int o = 0; o < NO; ++o) a[o] = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * o * K + (g << 3));
            if (tap != last_tap) {
                int dz, dy, dx;
                tap_offset(tap, k, dz, dy, dx);
                #pragma unroll
                for (int i = 0; i < FP; ++i) src[i] = pv[i] ? shifted(x, q[i], dz, dy, dx, pmask) : -1;
                last_tap = tap;
            }
            #pragma unroll
            for (int i = 0; i < FP; ++i)
                if (src[i] >= 0) b[i] = *reinterpret_cast<const bf16x8 *>(xp + src[i] * x.ctot + (c8 << 3));
        }
        #pragma unroll
        for (int o = 0; o < NO; ++o)
            #pragma unroll
            for (int i = 0; i < FP; ++i) acc[o][i] = mfma(a[o], b[i], acc[o][i]);
    }
    #pragma unroll
    for (int o = 0; o < NO; ++o)
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int oc = co0 + 16 * o + (grp << 2) + j;
            const bool sy = y.p && oc < y.c, s32 = y32.p && oc < y32.c;
            if (!sy && !s32) continue;                 // padded output rows
            const float bo = bias ? bias[oc] : 0.f;
            #pragma unroll
            for (int i = 0; i < FP; ++i) {
                if (!pv[i]) continue;
                const int64_t pb = p0 + 16 * i + col;
                float v = acc[o][i][j] + bo;
                if (relu) v = fmaxf(v, 0.f);
                if (sy) reinterpret_cast<bf16 *>(y.p)[pb * y.ctot + y.coff + oc] = (bf16)v;
                if (s32) {
                    float *out = reinterpret_cast<float *>(y32.p) + pb * y32.ctot + y32.coff + oc;
                    *out = accumulate ? *out + v : v;
                }
            }
        }
}

// 3x3x3 convolution on a brick of 16 (x) x 4 (y) x 4 ZW (z) output positions of
// one batch item, for tensors whose extents are multiples of the brick.  The
// brick's input halo (18 x 6 x (4 ZW + 2) positions) is staged in LDS one chunk
// of CT input channels at a time, so each input value is fetched from memory
// once per chunk instead of once per tap; the 27 taps then read their B
// fragments from LDS.  Wave w owns z-planes w ZW .. w ZW + ZW - 1 of the brick
// (4 ZW rows of 16 positions) and NO blocks of 16 output channels.  Layers with
// few input channels use ZW = 2, CT = 16: twice the MFMA work per staged halo at
// the same LDS size.  A staged position holds CT/8 16-byte chunks; the chunk
// index is XOR-swizzled with the position's x so that the 16 lanes of a
// fragment read (consecutive x, one chunk each) cover 256 distinct bytes and
// fall into different banks without padding.
constexpr int BX = 16, BY = 4;
constexpr int HX = BX + 2, HY = BY + 2;

// Workgroups are dealt to the 8 XCDs in turn by their linear id (x
// fastest).  This bijection on 0 .. n-1 maps the linear id to a position in
// the work order such that each XCD gets a contiguous run of it, so that
// neighbouring bricks, whose halos overlap, share an L2.
__device__ inline unsigned xcd_contiguous(unsigned lin, unsigned n)
{
    const unsigned x = lin & 7u, l = lin >> 3, q = n >> 3, r = n & 7u;
    return x * q + min(x, r) + l;
}

template <int NO, int ZW, int CT, bool DYR>
__global__ __launch_bounds__(256) void k_conv3_brick(sg_view x, const bf16 *__restrict__ W,
                                                     const float *__restrict__ bias, int pmask, int relu, sg_view y,
                                                     sg_view y32, int accumulate)
{
    constexpr int BZ = 4 * ZW, HZ = BZ + 2, HP = HX * HY * HZ, LROW = CT, NF = 4 * ZW;
    constexpr int NC = CT / 8, XSPAN = 16 / NC;           // chunks per position; positions per 256 bytes
    auto swz = [](int hx, int c8) { return c8 ^ ((hx / XSPAN) & (NC - 1)); };
    __shared__ __attribute__((aligned(16))) bf16 halo[HP * LROW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int nbx = x.w / BX, nby = x.h / BY, nbz = x.d / BZ;
    // work order: output-channel blocks of a brick adjacent, then bricks x-fastest
    const unsigned ncb = gridDim.y;
    const unsigned v = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * ncb);
    int bi = (int)(v / ncb);
    const int bxi = bi % nbx;
    bi /= nbx;
    const int byi = bi % nby;
    bi /= nby;
    const int bzi = bi % nbz;
    const int n = bi / nbz;
    const int X0 = bxi * BX, Y0 = byi * BY, Z0 = bzi * BZ;
    const int co0 = (int)(v % ncb) * 16 * NO;
    const int ci = x.c, K = 27 * ci;
    const bf16 *xp = reinterpret_cast<const bf16 *>(x.p) + x.coff;
    const bf16 *wrow = W + (int64_t)(co0 + col) * K;
    const bf16x8 zero = {};
    f32x4 acc[NO][NF];
    #pragma unroll
    for (int o = 0; o < NO; ++o)
        #pragma unroll
        for (int i = 0; i < NF; ++i) acc[o][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int c0 = 0; c0 < ci; c0 += CT) {
        const int gpt = min(CT, ci - c0) >> 3;           // 8-channel groups per tap in this chunk
        const int lgp = gpt == 1 ? 0 : (gpt == 2 ? 1 : 2);
        // stage the halo: every load of this thread is issued before the first
        // LDS store, so the chunk costs one memory latency, not one per element
        constexpr int PER = (HP * (CT / 8) + 255) / 256;
        bf16x8 hv[PER];
        int hdst[PER];
        #pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = (int)threadIdx.x + 256 * k;
            hdst[k] = -1;
            hv[k] = zero;
            if (e < (HP << lgp)) {
                const int hp = e >> lgp, c8 = e & (gpt - 1);
                const int hx = hp % HX, hy = (hp / HX) % HY, hz = hp / (HX * HY);
                int gx = X0 - 1 + hx, gy = Y0 - 1 + hy, gz = Z0 - 1 + hz;
                bool ok = true;
                if (gx < 0 || gx >= x.w) {
                    if (pmask & 1) gx = gx < 0 ? gx + x.w : gx - x.w;
                    else ok = false;
                }
                if (gy < 0 || gy >= x.h) {
                    if (pmask & 2) gy = gy < 0 ? gy + x.h : gy - x.h;
                    else ok = false;
                }
                if (gz < 0 || gz >= x.d) {
                    if (pmask & 4) gz = gz < 0 ? gz + x.d : gz - x.d;
                    else ok = false;
                }
                hdst[k] = hp * LROW + 8 * swz(hx, c8);
                if (ok)
                    hv[k] = *reinterpret_cast<const bf16x8 *>(
                        xp + ((((int64_t)n * x.d + gz) * x.h + gy) * x.w + gx) * x.ctot + c0 + 8 * c8);
            }
        }
        __syncthreads();                                  // previous chunk's fragment reads are done
        #pragma unroll
        for (int k = 0; k < PER; ++k)
            if (hdst[k] >= 0) *reinterpret_cast<bf16x8 *>(&halo[hdst[k]]) = hv[k];
        __syncthreads();
        if constexpr (DYR) {
            // The three dy taps of a (dz, dx, channel group) read the same
            // halo rows shifted by one: a lane loads the 6 rows its 4 output
            // rows need once and feeds them to three K blocks (dy = -1, 0, 1),
            // half the LDS fragment reads of one read per MFMA row and tap.
            // Super-block s gives lane group grp the combination q = 4 s + grp
            // of (dz, dx, c8); combinations past the last get zero weights.
            const int Q9 = 9 * gpt, nsb = (Q9 + 3) >> 2, lg = lgp;
            auto rows = [&](int s, bf16x8 (&R)[ZW][6]) {
                const int q = min(4 * s + grp, Q9 - 1);
                const int c8 = q & (gpt - 1), dzx = q >> lg;
                const int dz = dzx / 3, dx = dzx % 3;                 // 0..2: offsets + 1
                const int hx = col + dx;
                #pragma unroll
                for (int z = 0; z < ZW; ++z)
                    #pragma unroll
                    for (int r = 0; r < 6; ++r) {
                        const int hp = ((wave * ZW + z + dz) * HY + r) * HX + hx;
                        R[z][r] = *reinterpret_cast<const bf16x8 *>(&halo[hp * LROW + 8 * swz(hx, c8)]);
                    }
            };
            auto wts = [&](int s, bf16x8 (&A)[3][NO]) {
                const int q4 = 4 * s + grp, q = min(q4, Q9 - 1);
                const int c8 = q & (gpt - 1), dzx = q >> lg;
                const int dz = dzx / 3, dx = dzx % 3;
                #pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int tap = dz * 9 + d * 3 + dx;
                    #pragma unroll
                    for (int o = 0; o < NO; ++o) {
                        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * o * K + tap * ci + c0 + 8 * c8);
                        A[d][o] = q4 < Q9 ? v : zero;
                    }
                }
            };
            auto mma3 = [&](const bf16x8 (&R)[ZW][6], const bf16x8 (&A)[3][NO]) {
                #pragma unroll
                for (int d = 0; d < 3; ++d)
                    #pragma unroll
                    for (int o = 0; o < NO; ++o)
                        #pragma unroll
                        for (int i = 0; i < NF; ++i) acc[o][i] = mfma(A[d][o], R[i / 4][i % 4 + d], acc[o][i]);
            };
            bf16x8 R0[ZW][6], R1[ZW][6], A0[3][NO], A1[3][NO];
            rows(0, R0);
            wts(0, A0);
            int s = 0;
            for (; s + 2 <= nsb; s += 2) {
                rows(s + 1, R1);
                wts(s + 1, A1);
                mma3(R0, A0);
                const int sn = min(s + 2, nsb - 1);
                rows(sn, R0);
                wts(sn, A0);
                mma3(R1, A1);
            }
            if (s < nsb) mma3(R0, A0);
            continue;
        }
        // K blocks of 4 (tap, 8-channel group) pairs.  The full blocks run
        // unmasked; a last partial block (27 gpt not a multiple of 4) zeroes
        // the weights of its idle lanes.
        const int G = 27 * gpt, nfull = G >> 2, rem = G & 3, lg = lgp;
        auto fetch = [&](int g, bf16x8 (&a)[NO], bf16x8 (&b)[NF]) {
            const int tap = g >> lg, c8 = g & (gpt - 1);
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            #pragma unroll
            for (int o = 0; o < NO; ++o)
                a[o] = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * o * K + tap * ci + c0 + 8 * c8);
            #pragma unroll
            for (int i = 0; i < NF; ++i) {
                const int zl = wave * ZW + i / 4, yl = i % 4;
                const int hx = col + 1 + dx;
                const int hp = ((zl + 1 + dz) * HY + (yl + 1 + dy)) * HX + hx;
                b[i] = *reinterpret_cast<const bf16x8 *>(&halo[hp * LROW + 8 * swz(hx, c8)]);
            }
        };
        // two register sets in turn, so a block's MFMAs never wait for the
        // fetch issued after them; the fetch past the end re-reads a valid block
        auto mma = [&](const bf16x8 (&a)[NO], const bf16x8 (&b)[NF]) {
            #pragma unroll
            for (int o = 0; o < NO; ++o)
                #pragma unroll
                for (int i = 0; i < NF; ++i) acc[o][i] = mfma(a[o], b[i], acc[o][i]);
        };
        bf16x8 a[NO], b[NF], a1[NO], b1[NF];
        fetch(grp, a, b);
        int kb = 0;
        for (; kb + 2 <= nfull; kb += 2) {
            fetch(((kb + 1) << 2) + grp, a1, b1);
            mma(a, b);
            fetch((min(kb + 2, nfull - 1) << 2) + grp, a, b);
            mma(a1, b1);
        }
        if (kb < nfull) mma(a, b);
        if (rem) {
            const bool valid = grp < rem;
            fetch(valid ? (nfull << 2) + grp : G - 1, a, b);
            #pragma unroll
            for (int o = 0; o < NO; ++o) {
                if (!valid) a[o] = zero;
                #pragma unroll
                for (int i = 0; i < NF; ++i) acc[o][i] = mfma(a[o], b[i], acc[o][i]);
            }
        }
    }
    // A lane holds 4 consecutive output channels of each position: stored as
    // one 8-byte (BF16) or 16-byte (FP32) access when the slice allows it.
    const bool vy = y.p && ((y.ctot | y.coff) & 3) == 0;
    const bool v32 = y32.p && ((y32.ctot | y32.coff) & 3) == 0;
    #pragma unroll
    for (int o = 0; o < NO; ++o) {
        const int oc0 = co0 + 16 * o + (grp << 2);
        const int nbias = max(y.p ? y.c : 0, y32.p ? y32.c : 0);
        float bo[4];
        #pragma unroll
        for (int j = 0; j < 4; ++j) bo[j] = bias && oc0 + j < nbias ? bias[oc0 + j] : 0.f;
        const bool fy = vy && oc0 + 3 < y.c, f32 = v32 && oc0 + 3 < y32.c;
        #pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int zl = wave * ZW + i / 4, yl = i % 4;
            const int64_t pb = (((int64_t)n * x.d + Z0 + zl) * x.h + Y0 + yl) * x.w + X0 + col;
            f32x4 v;
            #pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = relu ? fmaxf(acc[o][i][j] + bo[j], 0.f) : acc[o][i][j] + bo[j];
            if (fy) {
                const bf16x4 q = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
                *reinterpret_cast<bf16x4 *>(reinterpret_cast<bf16 *>(y.p) + pb * y.ctot + y.coff + oc0) = q;
            } else if (y.p) {
                #pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (oc0 + j < y.c) reinterpret_cast<bf16 *>(y.p)[pb * y.ctot + y.coff + oc0 + j] = (bf16)v[j];
            }
            if (f32) {
                f32x4 *out = reinterpret_cast<f32x4 *>(reinterpret_cast<float *>(y32.p) + pb * y32.ctot + y32.coff + oc0);
                *out = accumulate ? *out + v : v;
            } else if (y32.p) {
                #pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (oc0 + j < y32.c) {
                        float *out = reinterpret_cast<float *>(y32.p) + pb * y32.ctot + y32.coff + oc0 + j;
                        *out = accumulate ? *out + v[j] : v[j];
                    }
            }
        }
    }
}

template <int NO, int ZW, int CT>
static void launch_brick(const sg_view *x, const void *w, const float *bias, int co, int pmask, int relu,
                         const sg_view &y, const sg_view &y32, int accumulate, hipStream_t st)
{
    const unsigned nb = (unsigned)((int64_t)x->n * (x->d / (4 * ZW)) * (x->h / BY) * (x->w / BX));
    // row reuse across the dy taps where it measured faster: one output block
    // (the full-resolution 16-channel layers: 364 -> 321 us on the 128 x 128 x
    // 512 box) and one-plane 32-channel chunks; the two-plane two-block forms
    // need 156-164 registers for it and lose occupancy (102 -> 143 us)
    constexpr bool dyr = NO == 1 || (ZW == 1 && CT == 32);
    hipLaunchKernelGGL((k_conv3_brick<NO, ZW, CT, dyr>), dim3(nb, co / (16 * NO)), dim3(256), 0, st, *x,
                       (const bf16 *)w, bias, pmask, relu, y, y32, accumulate);
}

// 1x1x1 convolution with few outputs (the network head): one position per
// lane, the weight rows read as wave-uniform vectors, FP32 dot products.  The
// layer moves ~3x more bytes than it computes, so it is written for HBM.
template <int NOUT>
__global__ __launch_bounds__(256) void k_conv1_small(sg_view x, const bf16 *__restrict__ W,
                                                     const float *__restrict__ bias, int relu, sg_view y, sg_view y32,
                                                     int accumulate)
{
    const int64_t P = npos(x);
    const int ci = x.c, g8 = ci >> 3;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        float acc[NOUT];
        #pragma unroll
        for (int o = 0; o < NOUT; ++o) acc[o] = bias ? bias[o] : 0.f;
        const bf16 *xr = reinterpret_cast<const bf16 *>(x.p) + p * x.ctot + x.coff;
        for (int g = 0; g < g8; ++g) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(xr + 8 * g);
            #pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                const bf16x8 w = *reinterpret_cast<const bf16x8 *>(W + (int64_t)o * ci + 8 * g);
                #pragma unroll
                for (int j = 0; j < 8; ++j) acc[o] = __builtin_fmaf((float)w[j], (float)v[j], acc[o]);
            }
        }
        #pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            float v = relu ? fmaxf(acc[o], 0.f) : acc[o];
            if (y.p && o < y.c) reinterpret_cast<bf16 *>(y.p)[p * y.ctot + y.coff + o] = (bf16)v;
            if (y32.p && o < y32.c) {
                float *out = reinterpret_cast<float *>(y32.p) + p * y32.ctot + y32.coff + o;
                *out = accumulate ? *out + v : v;
            }
        }
    }
}

// Master weights -> BF16 [co_pad][K] and the flipped transpose
// Wt[ci][tap' co8 + c] = W[c][tap ci + ci] with tap' the mirrored tap.
__global__ void k_weight_prep(const float *w32, int co, int ci, int k, bf16 *wb, bf16 *wt, int co_pad, int ci_pad)
{
    const int taps = k * k * k, K = taps * ci, co8 = (co + 7) & ~7, Kt = taps * co8;
    const int64_t n1 = (int64_t)co_pad * K, n2 = (int64_t)ci_pad * Kt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n1 + n2; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < n1) {
            const int o = (int)(e / K);
            wb[e] = (bf16)(o < co ? w32[e] : 0.f);
        } else {
            const int64_t f = e - n1;
            const int i = (int)(f / Kt), r = (int)(f % Kt);
            const int tp = r / co8, c = r % co8;
            const int tap = taps - 1 - tp;     // (dz,dy,dx) -> (-dz,-dy,-dx)
            wt[f] = (bf16)((i < ci && c < co) ? w32[(int64_t)c * K + (int64_t)tap * ci + i] : 0.f);
        }
    }
}

// ------------------------------------------------------ weight gradient
// dW[co][tap ci + c] = sum_p dy[p][co] x[p + off(tap)][c].  The contraction
// runs over positions, which are not contiguous in the channels-last tensors,
// so each workgroup stages a chunk of BPC positions in LDS transposed to
// position-fastest rows: dy for its 16 NOB output channels and, for every tap,
// the shifted x rows of its 16-channel input block.  The MFMA then reads
// A = dy^T (16 co x 32 positions) and B = x (32 positions x 16 channels) as
// 16-byte rows.  Wave w owns taps w, w + 4, ...; its accumulators stay in
// registers over all chunks of its position group (grid.x), and each group
// writes one partial sum per weight to ws[group][co_pad][K].
constexpr int BPC = 64;              // positions per staged chunk
constexpr int BROW = BPC + 8;        // LDS row length (bf16), padded against bank conflicts
constexpr int BTAPS = 7;             // taps per wave (27 taps over 4 waves)

template <int NOB>
__global__ __launch_bounds__(256) void k_conv_bwd_w(sg_view x, sg_view dy, int k, int pmask, int groups, int co_pad,
                                                    float *ws, float *wsb)
{
    __shared__ __attribute__((aligned(16))) bf16 xs[27][16][BROW];
    __shared__ __attribute__((aligned(16))) bf16 dyt[16 * NOB][BROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int ci = x.c, taps = k * k * k, K = taps * ci;
    const int co0 = blockIdx.y * 16 * NOB, c0 = blockIdx.z * 16;
    const int64_t P = npos(x);
    const int64_t nchunks = (P + BPC - 1) / BPC;
    const bf16 *xp = reinterpret_cast<const bf16 *>(x.p);
    const bf16 *dp = reinterpret_cast<const bf16 *>(dy.p);
    const bf16x8 zero = {};
    // staging roles: x rows: positions 2m, 2m+1 with m = (tid & 63) / 2, 8-channel
    // half tid & 1, taps congruent to tid / 64 modulo 4; the two positions of a
    // channel go to LDS as one 32-bit store
    const int xpair = (tid & 63) >> 1, xc8 = tid & 1, xtap0 = tid >> 6;
    const bool xcv = c0 + 8 * xc8 < ci;
    // dy rows: position tid / (2 NOB), 8-channel group tid % (2 NOB)
    const int dpos = tid / (2 * NOB), dc8 = tid % (2 * NOB);
    const int doc = co0 + 8 * dc8;
    f32x4 acc[BTAPS][NOB], accb[NOB];
    #pragma unroll
    for (int t = 0; t < BTAPS; ++t)
        #pragma unroll
        for (int o = 0; o < NOB; ++o) acc[t][o] = f32x4{0.f, 0.f, 0.f, 0.f};
    #pragma unroll
    for (int o = 0; o < NOB; ++o) accb[o] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the bias gradient is the weight gradient of an input channel of ones;
    // the wave with the fewest taps computes it in the first input-channel block
    const bool bias_wave = wsb && blockIdx.z == 0 && wave == taps % 4;
    bf16x8 ones;
    #pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = (bf16)1.f;

    constexpr int XT = 7;                                  // taps per thread: 27 taps over four residues
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += groups) {
        const int64_t pbase = ch * BPC;
        // every load of this thread for the chunk is issued before the barrier
        // and the LDS stores, so a chunk costs one memory latency
        bf16x8 xv[XT][2], dv = zero;
        #pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t p = pbase + 2 * xpair + h;
            const bool pv = p < P;
            const Pos q = decode(x, pv ? p : 0);
            #pragma unroll
            for (int i = 0; i < XT; ++i) {
                const int t = xtap0 + 4 * i;
                xv[i][h] = zero;
                if (t < taps && pv && xcv) {
                    int dz, dyo, dx;
                    tap_offset(t, k, dz, dyo, dx);
                    const int64_t src = shifted(x, q, dz, dyo, dx, pmask);
                    if (src >= 0)
                        xv[i][h] = *reinterpret_cast<const bf16x8 *>(xp + src * x.ctot + x.coff + c0 + 8 * xc8);
                }
            }
        }
        if (dpos < BPC) {
            const int64_t p = pbase + dpos;
            if (p < P && doc < dy.c) {
                dv = *reinterpret_cast<const bf16x8 *>(dp + p * dy.ctot + dy.coff + doc);
                #pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (doc + j >= dy.c) dv[j] = (bf16)0.f;
            }
        }
        __syncthreads();                                   // previous chunk's MFMA reads are done
        #pragma unroll
        for (int i = 0; i < XT; ++i) {
            const int t = xtap0 + 4 * i;
            if (t < taps)
                #pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bf16x2 pr = {xv[i][0][j], xv[i][1][j]};
                    *reinterpret_cast<bf16x2 *>(&xs[t][8 * xc8 + j][2 * xpair]) = pr;
                }
        }
        if (dpos < BPC)
            #pragma unroll
            for (int j = 0; j < 8; ++j) dyt[8 * dc8 + j][dpos] = dv[j];
        __syncthreads();
        #pragma unroll
        for (int ks = 0; ks < BPC / 32; ++ks) {
            bf16x8 a[NOB];
            #pragma unroll
            for (int o = 0; o < NOB; ++o) a[o] = *reinterpret_cast<const bf16x8 *>(&dyt[16 * o + col][32 * ks + 8 * grp]);
            #pragma unroll
            for (int ti = 0; ti < BTAPS; ++ti) {
                const int t = wave + 4 * ti;
                if (t < taps) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&xs[t][col][32 * ks + 8 * grp]);
                    #pragma unroll
                    for (int o = 0; o < NOB; ++o) acc[ti][o] = mfma(a[o], b, acc[ti][o]);
                }
            }
            if (bias_wave)
                #pragma unroll
                for (int o = 0; o < NOB; ++o) accb[o] = mfma(a[o], ones, accb[o]);
        }
    }
    if (bias_wave && col == 0)
        #pragma unroll
        for (int o = 0; o < NOB; ++o)
            #pragma unroll
            for (int j = 0; j < 4; ++j) wsb[(int64_t)blockIdx.x * co_pad + co0 + 16 * o + 4 * grp + j] = accb[o][j];
    // D[4 grp + j][col]: output channel co0 + 16 o + 4 grp + j, input channel c0 + col
    const int c = c0 + col;
    if (c >= ci) return;
    #pragma unroll
    for (int ti = 0; ti < BTAPS; ++ti) {
        const int t = wave + 4 * ti;
        if (t >= taps) continue;
        #pragma unroll
        for (int o = 0; o < NOB; ++o)
            #pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int oc = co0 + 16 * o + 4 * grp + j;
                ws[((int64_t)blockIdx.x * co_pad + oc) * K + (int64_t)t * ci + c] = acc[ti][o][j];
            }
    }
}

// Fixed-order sum of the per-group partials in two passes: slice s of the
// groups (g = s, s + S, ...) per thread and output, then the S slice sums.
__global__ void k_reduce_slices(const float *ws, int groups, int co_pad, int co, int K, int S, float *tmp)
{
    const int64_t n = (int64_t)co * K;
    const int s = blockIdx.y;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(e / K), kc = (int)(e % K);
        float acc = 0.f;
        for (int g = s; g < groups; g += S) acc += ws[((int64_t)g * co_pad + o) * K + kc];
        tmp[(int64_t)s * n + e] = acc;
    }
}

__global__ void k_reduce_final(const float *tmp, int S, int64_t n, float *dw)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int s = 0; s < S; ++s) acc += tmp[(int64_t)s * n + e];
        dw[e] = acc;
    }
}

// ------------------------------------------------------- element-wise
__global__ void k_relu_bwd_cast(sg_view dx, sg_view y, sg_view dyb)
{
    const int64_t n = npos(dx) * dx.c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / dx.c;
        const int c = (int)(e % dx.c);
        float g = reinterpret_cast<const float *>(dx.p)[p * dx.ctot + dx.coff + c];
        if (y.p && !((float)reinterpret_cast<const bf16 *>(y.p)[p * y.ctot + y.coff + c] > 0.f)) g = 0.f;
        reinterpret_cast<bf16 *>(dyb.p)[p * dyb.ctot + dyb.coff + c] = (bf16)g;
    }
}

__device__ inline int64_t flat(const sg_view &v, int n, int z, int y, int x)
{
    return (((int64_t)n * v.d + z) * v.h + y) * v.w + x;
}

__global__ void k_pool2_fwd(sg_view x, sg_view y)
{
    const int64_t n = npos(y) * y.c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / y.c;
        const int c = (int)(e % y.c);
        const Pos q = decode(y, p);
        float s = 0.f;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    s += (float)reinterpret_cast<const bf16 *>(x.p)[flat(x, q.n, 2 * q.z + dz, 2 * q.y + dy, 2 * q.x + dx) * x.ctot + x.coff + c];
        reinterpret_cast<bf16 *>(y.p)[p * y.ctot + y.coff + c] = (bf16)(0.125f * s);
    }
}

__global__ void k_pool2_bwd(sg_view dy, sg_view dx, int accumulate)
{
    const int64_t n = npos(dx) * dx.c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / dx.c;
        const int c = (int)(e % dx.c);
        const Pos q = decode(dx, p);
        const float g = 0.125f * reinterpret_cast<const float *>(dy.p)[flat(dy, q.n, q.z >> 1, q.y >> 1, q.x >> 1) * dy.ctot + dy.coff + c];
        float *o = reinterpret_cast<float *>(dx.p) + p * dx.ctot + dx.coff + c;
        *o = accumulate ? *o + g : g;
    }
}

__global__ void k_up2_fwd(sg_view x, sg_view y)
{
    const int64_t n = npos(y) * y.c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / y.c;
        const int c = (int)(e % y.c);
        const Pos q = decode(y, p);
        reinterpret_cast<bf16 *>(y.p)[p * y.ctot + y.coff + c] =
            reinterpret_cast<const bf16 *>(x.p)[flat(x, q.n, q.z >> 1, q.y >> 1, q.x >> 1) * x.ctot + x.coff + c];
    }
}

// 8-channel (16-byte) forms of the two sampling layers for channel-aligned views.
// One thread per coarse position and 8-channel group: the coarse chunk is read
// once and written to the 8 fine positions it covers.  Indices are 32-bit
// (the host checks that the coarse element count fits).
__global__ void k_up2_fwd8(sg_view x, sg_view y)
{
    const unsigned g8 = (unsigned)y.c >> 3;
    const unsigned n = (unsigned)npos(x) * g8;
    for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const unsigned p = e / g8, c = (e - p * g8) << 3;
        const unsigned px = p % (unsigned)x.w, t1 = p / (unsigned)x.w;
        const unsigned py = t1 % (unsigned)x.h, t2 = t1 / (unsigned)x.h;
        const unsigned pz = t2 % (unsigned)x.d, nb = t2 / (unsigned)x.d;
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const bf16 *>(x.p) +
                                                           (int64_t)p * x.ctot + x.coff + c);
        bf16 *yb = reinterpret_cast<bf16 *>(y.p) + y.coff + c;
        #pragma unroll
        for (int dz = 0; dz < 2; ++dz)
            #pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const int64_t row = (((int64_t)nb * y.d + 2 * pz + dz) * y.h + 2 * py + dy) * y.w + 2 * px;
                *reinterpret_cast<bf16x8 *>(yb + row * y.ctot) = v;
                *reinterpret_cast<bf16x8 *>(yb + (row + 1) * y.ctot) = v;
            }
    }
}

// Upsampling into a concatenation: y's first x.c channels are the nearest 2x
// upsampling of x, the remaining ones a copy of `skip` (same positions as y).
// One thread per fine position and 8-channel group of y, so that a position's
// whole row of y is written by adjacent lanes: full-line writes even where y
// interleaves the two parts per position.  32-bit indices (host-checked).
__global__ void k_up2_cat8(sg_view x, sg_view skip, sg_view y)
{
    const unsigned g8 = (unsigned)y.c >> 3, gx = (unsigned)x.c >> 3;
    const unsigned n = (unsigned)npos(y) * g8;
    for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const unsigned p = e / g8, g = e - p * g8;
        bf16x8 v;
        if (g < gx) {
            const unsigned fx = p % (unsigned)y.w, t1 = p / (unsigned)y.w;
            const unsigned fy = t1 % (unsigned)y.h, t2 = t1 / (unsigned)y.h;
            const unsigned fz = t2 % (unsigned)y.d, nb = t2 / (unsigned)y.d;
            const int64_t q = (((int64_t)nb * x.d + (fz >> 1)) * x.h + (fy >> 1)) * x.w + (fx >> 1);
            v = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const bf16 *>(x.p) + q * x.ctot + x.coff + 8 * g);
        } else {
            v = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const bf16 *>(skip.p) + (int64_t)p * skip.ctot +
                                                  skip.coff + 8 * (g - gx));
        }
        *reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16 *>(y.p) + (int64_t)p * y.ctot + y.coff + 8 * g) = v;
    }
}

// One thread per coarse position and 8-channel group; 32-bit indices (the
// host checks that the coarse element count fits).
__global__ void k_pool2_fwd8(sg_view x, sg_view y)
{
    const unsigned g8 = (unsigned)y.c >> 3;
    const unsigned n = (unsigned)npos(y) * g8;
    for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const unsigned p = e / g8, c = (e - p * g8) << 3;
        const unsigned px = p % (unsigned)y.w, t1 = p / (unsigned)y.w;
        const unsigned py = t1 % (unsigned)y.h, t2 = t1 / (unsigned)y.h;
        const unsigned pz = t2 % (unsigned)y.d, nb = t2 / (unsigned)y.d;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        #pragma unroll
        for (int dz = 0; dz < 2; ++dz)
            #pragma unroll
            for (int dy = 0; dy < 2; ++dy)
                #pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const int64_t q = (((int64_t)nb * x.d + 2 * pz + dz) * x.h + 2 * py + dy) * x.w + 2 * px + dx;
                    const bf16x8 v = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const bf16 *>(x.p) +
                                                                       q * x.ctot + x.coff + c);
                    #pragma unroll
                    for (int j = 0; j < 8; ++j) s[j] += (float)v[j];
                }
        bf16x8 o;
        #pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = (bf16)(0.125f * s[j]);
        *reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16 *>(y.p) + (int64_t)p * y.ctot + y.coff + c) = o;
    }
}

__global__ void k_up2_bwd(sg_view dy, sg_view dx, int accumulate)
{
    const int64_t n = npos(dx) * dx.c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / dx.c;
        const int c = (int)(e % dx.c);
        const Pos q = decode(dx, p);
        float s = 0.f;
        for (int dz = 0; dz < 2; ++dz)
            for (int dyy = 0; dyy < 2; ++dyy)
                for (int dxx = 0; dxx < 2; ++dxx)
                    s += reinterpret_cast<const float *>(dy.p)[flat(dy, q.n, 2 * q.z + dz, 2 * q.y + dyy, 2 * q.x + dxx) * dy.ctot + dy.coff + c];
        float *o = reinterpret_cast<float *>(dx.p) + p * dx.ctot + dx.coff + c;
        *o = accumulate ? *o + s : s;
    }
}

// MSE: per-workgroup partial sums (fixed order) then one workgroup.
__global__ __launch_bounds__(256) void k_mse(sg_view out, sg_view tgt, sg_view grad, double *partial)
{
    __shared__ double sh[256];
    const int64_t n = npos(out) * out.c;
    const double inv = 1.0 / (double)n;
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / out.c;
        const int c = (int)(e % out.c);
        const float d = reinterpret_cast<const float *>(out.p)[p * out.ctot + out.coff + c] -
                        reinterpret_cast<const float *>(tgt.p)[p * tgt.ctot + tgt.coff + c];
        reinterpret_cast<float *>(grad.p)[p * grad.ctot + grad.coff + c] = (float)(2.0 * d * inv);
        s += (double)d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] * inv;
}

__global__ void k_sum_partials(const double *partial, int n, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partial[i];
        *out = s;
    }
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[e];
        const float mi = b1 * m[e] + (1.f - b1) * gi;
        const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        w[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

struct Scale { float s[8]; };

__global__ void k_pack(const float *f, int nf, int nx, int ny, int nz, int x0, int y0, int z0, sg_view y, sg_view y32, int b,
                       Scale sc)
{
    const int64_t per = (int64_t)y.d * y.h * y.w;
    const int64_t n = per * y.c;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / y.c;
        const int c = (int)(e % y.c);
        const int x = (int)(p % y.w), yy = (int)((p / y.w) % y.h), z = (int)(p / ((int64_t)y.w * y.h));
        float v = 0.f;
        if (c < nf) {
            const int gx = (x0 + x) % nx, gy = (y0 + yy) % ny, gz = (z0 + z) % nz;
            v = f[(int64_t)c * nx * ny * nz + gx + (int64_t)nx * (gy + (int64_t)ny * gz)] / sc.s[c];
        }
        const int64_t pp = (int64_t)b * per + p;
        reinterpret_cast<bf16 *>(y.p)[pp * y.ctot + y.coff + c] = (bf16)v;
        if (y32.p && c < y32.c) reinterpret_cast<float *>(y32.p)[pp * y32.ctot + y32.coff + c] = v;
    }
}

// Position-per-lane form of k_pack for an 8-channel BF16 view (the network
// input): the nf planar fields are read coalesced, one 16-byte BF16 row and
// (optionally) the FP32 row are written per position.
__global__ void k_pack8(const float *f, int nf, int nx, int ny, int nz, int x0, int y0, int z0, sg_view y, sg_view y32,
                        int b, Scale sc)
{
    const int64_t per = (int64_t)y.d * y.h * y.w;
    const int64_t nxyz = (int64_t)nx * ny * nz;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < per; p += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(p % y.w), yy = (int)((p / y.w) % y.h), z = (int)(p / ((int64_t)y.w * y.h));
        const int gx = (x0 + x) % nx, gy = (y0 + yy) % ny, gz = (z0 + z) % nz;
        const int64_t src = gx + (int64_t)nx * (gy + (int64_t)ny * gz);
        float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < nf; ++c) v[c] = f[(int64_t)c * nxyz + src] / sc.s[c];
        bf16x8 o;
        #pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = (bf16)v[j];
        const int64_t pp = (int64_t)b * per + p;
        *reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16 *>(y.p) + pp * y.ctot + y.coff) = o;
        if (y32.p)
            for (int c = 0; c < y32.c; ++c) reinterpret_cast<float *>(y32.p)[pp * y32.ctot + y32.coff + c] = v[c];
    }
}

__global__ void k_unpack(sg_view x, int b, float *f, int nf, Scale sc)
{
    const int64_t per = (int64_t)x.d * x.h * x.w;
    const int64_t n = per * nf;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / per);
        const int64_t p = e % per;
        f[e] = reinterpret_cast<const float *>(x.p)[((int64_t)b * per + p) * x.ctot + x.coff + c] * sc.s[c];
    }
}

__global__ void k_lift(const float *pred, int64_t n, const float *pR, const float *pB, float cs2R, float cs2B,
                       float p_in, double *out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float v = fminf(1.f, fmaxf(-1.f, pred[e]));
        const float p = pR ? pR[e] * cs2R + pB[e] * cs2B : p_in;
        out[e] = (double)(0.5f * p * (1.f + v) / cs2R);
        out[n + e] = (double)(0.5f * p * (1.f - v) / cs2B);
        out[2 * n + e] = (double)pred[n + e];
        out[3 * n + e] = (double)pred[2 * n + e];
        out[4 * n + e] = (double)pred[3 * n + e];
    }
}

inline unsigned grid_for(int64_t n, int block = 256)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 65536));
}

inline bool ok_view(const sg_view *v) { return v && v->p && v->n > 0 && v->d > 0 && v->h > 0 && v->w > 0 && v->c > 0 && v->coff >= 0 && v->coff + v->c <= v->ctot; }
inline bool mfma_view(const sg_view *v) { return ok_view(v) && v->c % 8 == 0 && v->ctot % 8 == 0 && v->coff % 8 == 0; }
inline bool same_pos(const sg_view *a, const sg_view *b) { return a->n == b->n && a->d == b->d && a->h == b->h && a->w == b->w; }

int status() { return hipGetLastError() == hipSuccess ? SG_OK : SG_EDEVICE; }

// Scratch of the no-allocation weight gradient: a file-scope device array,
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address of each GPU's copy is looked up once, with
// that GPU current, and kept.
static __device__ __align__(256) float scratch[SG_NOALLOC_SCRATCH_BYTES / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(float **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SG_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SG_EDEVICE;
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SG_OK;
}

}  // namespace sg

using namespace sg;

extern "C" {

int sg_conv3d_fwd(const sg_view *x, const void *w, const float *bias, int32_t co, int32_t k, int32_t periodic_mask,
                  int32_t relu, const sg_view *y, const sg_view *y32, int32_t accumulate, void *hip_stream)
{
    if (!mfma_view(x) || !w || co <= 0 || co % 16 || (k != 1 && k != 3)) return SG_EINVAL;
    if (!y && !y32) return SG_EINVAL;
    if (y && (!ok_view(y) || !same_pos(x, y) || y->c > co)) return SG_EINVAL;
    if (y32 && (!ok_view(y32) || !same_pos(x, y32) || y32->c > co)) return SG_EINVAL;
    const sg_view none = {};
    const int64_t P = (int64_t)x->n * x->d * x->h * x->w;
    if (k == 3 && x->w % BX == 0 && x->h % BY == 0 && x->d % 4 == 0) {
        hipStream_t st = (hipStream_t)hip_stream;
        const sg_view yv = y ? *y : none, y32v = y32 ? *y32 : none;
        const bool deep = x->c % 32 != 0 && x->d % 8 == 0;   // few or odd channel counts: two planes per wave
        // a 32-channel chunk stages 1, 2 or 4 eight-channel groups per position;
        // an input channel count of 24 mod 32 would leave a last chunk of 3
        // groups, so those layers stage 16-channel chunks
        const bool ct16 = x->c % 32 == 24;
        // two planes per wave also for 32-channel chunks when that still leaves
        // at least 512 workgroups (large layers: less halo per output; measured
        // on the U-Net, smaller layers lose from the fewer workgroups)
        const bool big = x->d % 8 == 0 && P / (BX * BY * 8) * (co / 32) >= 512;
        if (co % 32 == 0) {
            if (deep) launch_brick<2, 2, 16>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
            else if (ct16) launch_brick<2, 1, 16>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
            else if (big) launch_brick<2, 2, 32>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
            else launch_brick<2, 1, 32>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
        } else {
            if (deep) launch_brick<1, 2, 16>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
            else if (ct16) launch_brick<1, 1, 16>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
            else launch_brick<1, 1, 32>(x, w, bias, co, periodic_mask, relu, yv, y32v, accumulate, st);
        }
        return status();
    }
    const int nout = std::max(y ? y->c : 0, y32 ? y32->c : 0);
    if (k == 1 && nout <= 4 && x->c <= 64) {
        hipLaunchKernelGGL(k_conv1_small<4>, dim3(grid_for(P)), dim3(256), 0, (hipStream_t)hip_stream, *x,
                           (const bf16 *)w, bias, relu, y ? *y : none, y32 ? *y32 : none, accumulate);
        return status();
    }
    const unsigned gx = (unsigned)((P + 64 * FP - 1) / (64 * FP));
    if (co % 32 == 0)
        hipLaunchKernelGGL(k_conv_fwd<2>, dim3(gx, co / 32), dim3(256), 0, (hipStream_t)hip_stream, *x, (const bf16 *)w,
                           bias, k, periodic_mask, relu, y ? *y : none, y32 ? *y32 : none, accumulate);
    else
        hipLaunchKernelGGL(k_conv_fwd<1>, dim3(gx, co / 16), dim3(256), 0, (hipStream_t)hip_stream, *x, (const bf16 *)w,
                           bias, k, periodic_mask, relu, y ? *y : none, y32 ? *y32 : none, accumulate);
    return status();
}

int sg_weight_prep(const float *w32, int32_t co, int32_t ci, int32_t k, void *w_bf16, void *wt_bf16, int32_t co_pad,
                   int32_t ci_pad, void *hip_stream)
{
    if (!w32 || !w_bf16 || !wt_bf16 || co <= 0 || ci <= 0 || co_pad < co || ci_pad < ci || co_pad % 16 || ci_pad % 16 ||
        (k != 1 && k != 3))
        return SG_EINVAL;
    const int taps = k * k * k;
    const int64_t n = (int64_t)co_pad * taps * ci + (int64_t)ci_pad * taps * ((co + 7) & ~7);
    hipLaunchKernelGGL(k_weight_prep, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, w32, co, ci, k,
                       (bf16 *)w_bf16, (bf16 *)wt_bf16, co_pad, ci_pad);
    return status();
}

struct BwdPlan { int nob, groups, co_pad, cblocks, K, S; int64_t ws_floats, bias_off, tmp_off, tmpb_off; };

static BwdPlan bwd_plan(const sg_view *dy, int ci, int k)
{
    BwdPlan b;
    b.co_pad = (dy->c + 15) & ~15;
    b.nob = b.co_pad % 32 == 0 ? 2 : 1;
    b.cblocks = (ci + 15) / 16;
    b.K = k * k * k * ci;
    const int64_t P = (int64_t)dy->n * dy->d * dy->h * dy->w;
    const int64_t nchunks = (P + BPC - 1) / BPC;
    const int64_t yz = (int64_t)(b.co_pad / (16 * b.nob)) * b.cblocks;
    int64_t g = std::max<int64_t>(1, std::min<int64_t>(nchunks, (1024 + yz - 1) / yz));
    // keep the partial sums within 64 Mi floats
    g = std::max<int64_t>(1, std::min<int64_t>(g, ((int64_t)1 << 26) / ((int64_t)b.co_pad * b.K)));
    b.groups = (int)g;
    b.S = (int)std::min<int64_t>(16, g);
    b.bias_off = g * b.co_pad * b.K;
    b.tmp_off = b.bias_off + g * b.co_pad;
    b.tmpb_off = b.tmp_off + (int64_t)b.S * b.co_pad * b.K;
    b.ws_floats = b.tmpb_off + (int64_t)b.S * b.co_pad;
    return b;
}

int64_t sg_conv3d_bwd_weight_ws(const sg_view *dy, int32_t ci, int32_t k)
{
    if (!ok_view(dy) || ci <= 0 || (k != 1 && k != 3)) return -1;
    return bwd_plan(dy, ci, k).ws_floats * (int64_t)sizeof(float);
}

static bool bwd_weight_args(const sg_view *x, const sg_view *dy, int32_t k, const float *dw)
{
    return mfma_view(x) && ok_view(dy) && dy->ctot % 8 == 0 && dy->coff % 8 == 0 && dy->c <= 256 && same_pos(x, dy) &&
           dw && (k == 1 || k == 3);
}

// The weight-gradient kernels with the per-group partial sums in ws (at least
// b.ws_floats floats); shared by the workspace and the no-allocation entries.
static int bwd_weight_launch(const sg_view *x, const sg_view *dy, int32_t k, int32_t periodic_mask, float *dw,
                             float *db, float *ws, const BwdPlan &b, hipStream_t st)
{
    const int ci = x->c, co = dy->c;
    const dim3 grid(b.groups, b.co_pad / (16 * b.nob), b.cblocks);
    float *wsb = db ? ws + b.bias_off : nullptr;
    if (b.nob == 2)
        hipLaunchKernelGGL(k_conv_bwd_w<2>, grid, dim3(256), 0, st, *x, *dy, k, periodic_mask, b.groups, b.co_pad, ws,
                           wsb);
    else
        hipLaunchKernelGGL(k_conv_bwd_w<1>, grid, dim3(256), 0, st, *x, *dy, k, periodic_mask, b.groups, b.co_pad, ws,
                           wsb);
    const int64_t nw = (int64_t)co * b.K;
    hipLaunchKernelGGL(k_reduce_slices, dim3(grid_for(nw), b.S), dim3(256), 0, st, (const float *)ws, b.groups, b.co_pad,
                       co, b.K, b.S, ws + b.tmp_off);
    hipLaunchKernelGGL(k_reduce_final, dim3(grid_for(nw)), dim3(256), 0, st, (const float *)(ws + b.tmp_off), b.S, nw, dw);
    if (db) {
        hipLaunchKernelGGL(k_reduce_slices, dim3(grid_for(co), b.S), dim3(256), 0, st, (const float *)wsb, b.groups,
                           b.co_pad, co, 1, b.S, ws + b.tmpb_off);
        hipLaunchKernelGGL(k_reduce_final, dim3(grid_for(co)), dim3(256), 0, st, (const float *)(ws + b.tmpb_off), b.S,
                           (int64_t)co, db);
    }
    (void)ci;
    return status();
}

int sg_conv3d_bwd_weight(const sg_view *x, const sg_view *dy, int32_t k, int32_t periodic_mask, float *dw, float *db,
                         float *ws, int64_t ws_bytes, void *hip_stream)
{
    if (!bwd_weight_args(x, dy, k, dw) || !ws) return SG_EINVAL;
    const BwdPlan b = bwd_plan(dy, x->c, k);
    if (ws_bytes < b.ws_floats * (int64_t)sizeof(float)) return SG_EINVAL;
    return bwd_weight_launch(x, dy, k, periodic_mask, dw, db, ws, b, (hipStream_t)hip_stream);
}

int sg_conv3d_bwd_weight_noalloc(const sg_view *x, const sg_view *dy, int32_t k, int32_t periodic_mask, float *dw,
                                 float *db, void *hip_stream)
{
    if (!bwd_weight_args(x, dy, k, dw)) return SG_EINVAL;
    const BwdPlan b = bwd_plan(dy, x->c, k);
    if (b.ws_floats * (int64_t)sizeof(float) > SG_NOALLOC_SCRATCH_BYTES) return SG_EINVAL;
    float *ws = nullptr;
    const int rc = scratch_on_current_device(&ws);
    if (rc != SG_OK) return rc;
    return bwd_weight_launch(x, dy, k, periodic_mask, dw, db, ws, b, (hipStream_t)hip_stream);
}

int sg_relu_bwd_cast(const sg_view *dx, const sg_view *y, const sg_view *dyb, void *hip_stream)
{
    if (!ok_view(dx) || !ok_view(dyb) || !same_pos(dx, dyb) || dx->c != dyb->c) return SG_EINVAL;
    if (y && (!ok_view(y) || !same_pos(dx, y) || y->c != dx->c)) return SG_EINVAL;
    const sg_view none = {};
    const int64_t n = (int64_t)dx->n * dx->d * dx->h * dx->w * dx->c;
    hipLaunchKernelGGL(k_relu_bwd_cast, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *dx, y ? *y : none,
                       *dyb);
    return status();
}

static bool half_of(const sg_view *big, const sg_view *small)
{
    return big->n == small->n && big->d == 2 * small->d && big->h == 2 * small->h && big->w == 2 * small->w &&
           big->c == small->c;
}

int sg_pool2_fwd(const sg_view *x, const sg_view *y, void *hip_stream)
{
    if (!ok_view(x) || !ok_view(y) || !half_of(x, y)) return SG_EINVAL;
    const int64_t n = (int64_t)y->n * y->d * y->h * y->w * y->c;
    if (mfma_view(x) && mfma_view(y) && n / 8 < (int64_t)1 << 31)
        hipLaunchKernelGGL(k_pool2_fwd8, dim3(grid_for(n / 8)), dim3(256), 0, (hipStream_t)hip_stream, *x, *y);
    else
        hipLaunchKernelGGL(k_pool2_fwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *x, *y);
    return status();
}

int sg_pool2_bwd(const sg_view *dy, const sg_view *dx, int32_t accumulate, void *hip_stream)
{
    if (!ok_view(dy) || !ok_view(dx) || !half_of(dx, dy)) return SG_EINVAL;
    const int64_t n = (int64_t)dx->n * dx->d * dx->h * dx->w * dx->c;
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *dy, *dx, accumulate);
    return status();
}

int sg_up2_cat_fwd(const sg_view *x, const sg_view *skip, const sg_view *y, void *hip_stream)
{
    if (!mfma_view(x) || !mfma_view(skip) || !mfma_view(y)) return SG_EINVAL;
    if (y->n != x->n || y->d != 2 * x->d || y->h != 2 * x->h || y->w != 2 * x->w) return SG_EINVAL;
    if (!same_pos(y, skip) || y->c != x->c + skip->c) return SG_EINVAL;
    const int64_t n = (int64_t)y->n * y->d * y->h * y->w * (y->c / 8);
    if (n >= (int64_t)1 << 31) return SG_EINVAL;
    hipLaunchKernelGGL(k_up2_cat8, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *x, *skip, *y);
    return status();
}

int sg_up2_fwd(const sg_view *x, const sg_view *y, void *hip_stream)
{
    if (!ok_view(x) || !ok_view(y) || !half_of(y, x)) return SG_EINVAL;
    const int64_t n = (int64_t)y->n * y->d * y->h * y->w * y->c;
    if (mfma_view(x) && mfma_view(y) && n / 64 < (int64_t)1 << 31)
        hipLaunchKernelGGL(k_up2_fwd8, dim3(grid_for(n / 64)), dim3(256), 0, (hipStream_t)hip_stream, *x, *y);
    else
        hipLaunchKernelGGL(k_up2_fwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *x, *y);
    return status();
}

int sg_up2_bwd(const sg_view *dy, const sg_view *dx, int32_t accumulate, void *hip_stream)
{
    if (!ok_view(dy) || !ok_view(dx) || !half_of(dy, dx)) return SG_EINVAL;
    const int64_t n = (int64_t)dx->n * dx->d * dx->h * dx->w * dx->c;
    hipLaunchKernelGGL(k_up2_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *dy, *dx, accumulate);
    return status();
}

int sg_mse(const sg_view *out, const sg_view *target, const sg_view *grad, double *loss, void *hip_stream)
{
    if (!ok_view(out) || !ok_view(target) || !ok_view(grad) || !loss || !same_pos(out, target) ||
        !same_pos(out, grad) || out->c != target->c || out->c != grad->c)
        return SG_EINVAL;
    const int nb = 256;
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, (hipStream_t)hip_stream, *out, *target, *grad, loss + 1);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, (hipStream_t)hip_stream, (const double *)(loss + 1), nb, loss);
    return status();
}

int sg_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2, float eps,
            int64_t step, void *hip_stream)
{
    if (!w || !g || !m || !v || n <= 0 || step < 1) return SG_EINVAL;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, w, g, m, v, n, lr, beta1, beta2,
                       eps, c1, c2);
    return status();
}

static bool make_scale(const float *scale, int nf, Scale &sc)
{
    if (nf > 8) return false;
    for (int c = 0; c < 8; ++c) sc.s[c] = 1.0f;
    if (scale)
        for (int c = 0; c < nf; ++c) {
            if (!(scale[c] != 0.0f)) return false;
            sc.s[c] = scale[c];
        }
    return true;
}

int sg_pack(const float *f, int32_t nf, int32_t nx, int32_t ny, int32_t nz, int32_t x0, int32_t y0, int32_t z0,
            const float *scale, const sg_view *y, const sg_view *y32, int32_t b, void *hip_stream)
{
    Scale sc;
    if (!f || !ok_view(y) || nf <= 0 || nf > y->c || b < 0 || b >= y->n || x0 < 0 || y0 < 0 || z0 < 0 ||
        !make_scale(scale, nf, sc))
        return SG_EINVAL;
    if (y32 && (!ok_view(y32) || !same_pos(y, y32))) return SG_EINVAL;
    const sg_view none = {};
    if (y->c == 8 && mfma_view(y) && (!y32 || y32->c <= 8)) {
        const int64_t per = (int64_t)y->d * y->h * y->w;
        hipLaunchKernelGGL(k_pack8, dim3(grid_for(per)), dim3(256), 0, (hipStream_t)hip_stream, f, nf, nx, ny, nz, x0, y0,
                           z0, *y, y32 ? *y32 : none, b, sc);
        return status();
    }
    const int64_t n = (int64_t)y->d * y->h * y->w * y->c;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, f, nf, nx, ny, nz, x0, y0, z0,
                       *y, y32 ? *y32 : none, b, sc);
    return status();
}

int sg_unpack(const sg_view *x32, int32_t b, const float *scale, float *f, int32_t nf, void *hip_stream)
{
    Scale sc;
    if (!ok_view(x32) || !f || nf <= 0 || nf > x32->c || b < 0 || b >= x32->n || !make_scale(scale, nf, sc))
        return SG_EINVAL;
    const int64_t n = (int64_t)x32->d * x32->h * x32->w * nf;
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, *x32, b, f, nf, sc);
    return status();
}

int sg_lift(const float *pred, int64_t n, const float *rhoR_prev, const float *rhoB_prev, double cs2R, double cs2B,
            double p_in, double *out, void *hip_stream)
{
    if (!pred || !out || n <= 0 || !(cs2R > 0.0) || !(cs2B > 0.0) || (!rhoR_prev) != (!rhoB_prev) ||
        (!rhoR_prev && !(p_in > 0.0)))
        return SG_EINVAL;
    hipLaunchKernelGGL(k_lift, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, pred, n, rhoR_prev, rhoB_prev,
                       (float)cs2R, (float)cs2B, (float)p_in, out);
    return status();
}

}  // extern "C"
