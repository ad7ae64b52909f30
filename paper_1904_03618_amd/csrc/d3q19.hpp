// d3q19.hpp -- lattice constants, storage codecs and per-case parameters of the
// gfx950 implementation of the improved 3D colour-gradient LB model
// (Wen, Li, Yu & Luo, arXiv 1904.03618).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbcg.h"

namespace lbcg {

constexpr int Q = 19;

// Eq. (5): D3Q19 velocities, i = 0..18.  Every use sits in a fully unrolled
// loop, so these fold to immediates.
__host__ __device__ constexpr int ex(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int ey(int i)
{
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int ez(int i)
{
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
// velocity class: 0 rest, 1 axis (|e|^2 = 1), 2 face diagonal (|e|^2 = 2)
__host__ __device__ constexpr int ecls(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : 2); }
// the direction with e_opp = -e_i (pairs (1,2), (3,4), ... (17,18))
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }

// Level formats.  PAIR: every direction stores its red and blue deviation
// (Storage::P per node and direction).  COMPACT: direction 0 stores the pair,
// directions 1-18 store only the total deviation t_i = sum_k d_i^k
// (Storage::T), and each writer stores, besides its densities, the data from
// which a puller rebuilds the red share of any of its values exactly as the
// recoloring (Eq. 10-11) defines it: d_i^R = (rho_R/rho) t_i + seg_i + cr_c,
// with seg_i = e_i . g on the axes and kDiagSeg e_i . g on the diagonals
// (g = beta rho_R rho_B p n / (6 rho^2)), cr the class share of the rest
// state and of the densities' FP32 remainders (cr on the diagonals is half
// the axis value, as phi^k is).  A COMPACT level moves 20 + 7 words per node
// and level instead of 38 + 2 (20 population values plus 7 FP32 words).
constexpr int LV_PAIR = 0, LV_COMPACT = 1;
constexpr float kDiagSeg = 0.35355339059327378f;        // (1/2) cos 45 deg

// Population storage.  Every format keeps deviations d = f - rho_k phi_i^k
// from the rest state of the node that wrote the value (rho_k: that node's
// colour density, kept per node in FP32), scaled by 2^s for FP16.  The node's
// own stored density plus the small deviations carries the populations with
// well beyond FP32 resolution, so rounding does not bias the colour masses.
// The red and blue values of one direction at one node are stored side by
// side, so one 2-element access moves both colours.
template <class T> struct Pair { T r, b; };

template <int ST> struct Storage;
template <> struct Storage<LBCG_FP32> {
    using T = float;
    using P = Pair<T>;
    __device__ static float dec(T v, float) { return v; }
    __device__ static T enc(float d, float) { return d; }
};
template <> struct Storage<LBCG_FP16S> {
    using T = _Float16;
    using P = Pair<T>;
    // the scale is a power of two, so the product is exact and one
    // mixed-precision FMA (conversion and multiply fused) gives the same value
    __device__ static float dec(T v, float inv_scale) { return __builtin_fmaf((float)v, inv_scale, 0.0f); }
    __device__ static T enc(float d, float scale) { return (T)(d * scale); }
};
template <> struct Storage<LBCG_BF16S> {
    using T = __bf16;
    using P = Pair<T>;
    // BF16's exponent range needs no scale (the handle's scale is 1)
    __device__ static float dec(T v, float) { return (float)v; }
    __device__ static T enc(float d, float) { return (T)d; }
};

// Cache policy of the population streams: loads are non-temporal, so that a
// pass's stream does not displace the reused per-node arrays (aux stencil,
// stored densities) from L2; stores are ordinary, so that the level just
// written is still in the caches when the next pass reads it (measured: FP16S
// step 152 -> 142 us, FP32 228 -> 221 us on the 128^3 benchmark).

// Buffer-resource access.  A resource (base, size in bytes) is uniform over
// the wavefront and lives in scalar registers; each lane supplies only a
// 32-bit byte offset, so a pull costs no 64-bit address arithmetic per lane.
// Accesses beyond the size read zero and drop writes.  Cache policy: 2 marks a
// streamed, non-temporal access; 0 is the default.
constexpr int CP_DEFAULT = 0, CP_STREAM = 2;

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base, uint64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)(uint32_t)bytes, 0x00020000);
}

template <class T, int CP>
__device__ inline T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    if constexpr (sizeof(T) == 2) {
        const unsigned short v = __builtin_amdgcn_raw_buffer_load_b16(r, (int)byte_off, 0, CP);
        return __builtin_bit_cast(T, v);
    } else if constexpr (sizeof(T) == 4) {
        const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, CP);
        return __builtin_bit_cast(T, v);
    } else if constexpr (sizeof(T) == 8) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, CP);
        return __builtin_bit_cast(T, v);
    } else {
        static_assert(sizeof(T) == 16, "buffer element size");
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, CP);
        return __builtin_bit_cast(T, v);
    }
}

// The same with a wave-uniform byte offset soff added by the hardware (a
// scalar operand, no per-lane address arithmetic).
template <class T, int CP>
__device__ inline T buf_ld_so(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, uint32_t soff)
{
    if constexpr (sizeof(T) == 2) {
        const unsigned short v = __builtin_amdgcn_raw_buffer_load_b16(r, (int)byte_off, (int)soff, CP);
        return __builtin_bit_cast(T, v);
    } else if constexpr (sizeof(T) == 4) {
        const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, (int)soff, CP);
        return __builtin_bit_cast(T, v);
    } else {
        static_assert(sizeof(T) == 8, "buffer element size");
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, (int)soff, CP);
        return __builtin_bit_cast(T, v);
    }
}

template <class T, int CP>
__device__ inline void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, T val)
{
    if constexpr (sizeof(T) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, val), r, (int)byte_off, 0, CP);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, val), r, (int)byte_off, 0, CP);
    } else if constexpr (sizeof(T) == 8) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, val), r, (int)byte_off, 0, CP);
    } else {
        static_assert(sizeof(T) == 16, "buffer element size");
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, val), r, (int)byte_off, 0, CP);
    }
}


// Per-case constants, derived on the host in FP64 and rounded once to FP32.
struct DevCase {
    int nx, ny, nz, wall;        // wall: -1 none, else the wall axis
    int N, plane;                // nodes; nodes of one wall plane
    int improved;
    int NS;                      // stride of the population arrays: N rounded up to 64 nodes
    int64_t pop_off;             // first population element of the case
    int64_t node_off;            // first node of the case in per-node arrays
    int64_t ghost_off;           // first ghost entry (2 planes) of the case
    float rin_inv[2];            // 1 / rho_k^in
    float cs2[2];                // (c_s^k)^2 = (1 - alpha_k)/2
    float qc[2];                 // 1 - 3 (c_s^k)^2
    float phi[2][3];             // phi^k for rest / axis / diagonal (Eq. 13)
    float tauR, tauB, s1, s2, s3, t2, t3, delta;   // Eq. (52) and its parabolas
    float s_e, s_q, s_pi;        // 1/tau_e, 1/tau_q, 1/tau_pi (Eq. 44)
    float Asum, beta;            // A_R + A_B; recoloring beta
    float F[3], g[3], rho_ref;   // force density = F + (rho - rho_ref) g
    float cot[2];                // cot(theta) of the low / high wall
    float neg_tol[2];            // stability check: rho_k < neg_tol[k] is unstable
    float uw[2][3];              // velocity of the low / high wall (tangential)
    float wg[2][2];              // wall gain per colour for axis / diagonal links, per unit rho_k (e_i . U_w)
    int moving;                  // 1 when a wall velocity is nonzero
    float c16;                   // rows 16-18 of m^eq: coefficient of rho (u_a^2 + u_b^2)
};

struct StepArgs {
    const void *fin;             // populations at level t
    void *fout;                  // populations at level t+1
    float4 *aux;                 // per node: rho^N, Qbar_x, Qbar_y, Qbar_z (level t)
    float4 *ghost;               // per wall-plane node: same fields one layer beyond the wall
    const float2 *rho_prev;      // rho_R, rho_B the writers of fin stored with their values
    float2 *rho_cur;             // rho_R, rho_B stored with fout
    const float4 *dsc_prev;      // compact levels: the writers' recoloring data of fin
    float4 *dsc_cur;             //   (rho_R/rho, g_x, g_y, g_z) stored with fout
    const float *crs_prev;       //   and the axis-class rest-share term
    float *crs_cur;
    float *wallq;                // per ghost entry: sum_k rho_k (1 - 3 c_s^k^2) of the first layer
    const DevCase *cases;
    const int2 *tiles;           // (case, first node) per tile
    int ntiles;
    float scale, inv_scale;
};

}  // namespace lbcg
