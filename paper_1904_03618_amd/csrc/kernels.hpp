// kernels.hpp -- gfx950 kernels of one time step of the improved 3D
// colour-gradient MRT lattice Boltzmann model (Wen, Li, Yu & Luo).
//
// A step at level t is either one launch of k_fused (below: z-marching
// tiles, the phase-field halo in LDS; cases with walls, if any, on z), or the
// two-pass form, three launches over all tiles of all cases:
//   k_aux     pull the 38 populations, moments (Eq. 4), phase field rho^N
//             (text after Eq. 8) and Qbar = u sum_k rho_k (1 - 3 c_s^k^2)
//             (Eq. 46-49) -> aux
//   k_ghost   ghost layer one node beyond each wall (wetting rule for rho^N,
//             odd reflection for Qbar)
//   k_collide pull the 38 populations again, colour gradient and Q_alpha from
//             the aux stencil (Eq. 49), tau_v (Eq. 52), the two-colour MRT
//             collision in moment space (Eq. 41-45, 53 and the body force),
//             recoloring (Eq. 10-11) and store at the node's own slots: the
//             next step's pull completes the streaming.
// All population arithmetic runs on deviations from the local rest state
// (see Storage): with S_k the density a node stored at the previous level and
// R_k its new density, the pulled f_i^k = rho_k(src) phi_i^k + d_i^k enter as
// h_i = sum_k [(rho_k(src) - S_k) phi_i^k + d_i^k], R_k = S_k + sum of the
// colour's h terms, and g_i = f_i - sum_k R_k phi_i^k; the rest state is
// isotropic, so its moments are known in closed form and never rounded.
// The colour gradient at level t needs the level-t densities of all 18
// neighbours, so in the two-pass form the moments pass must finish before the
// collision pass.  Levels are stored as colour pairs or, with the fused step,
// in the compact format of d3q19.hpp (totals plus the writers' recoloring
// data).
#pragma once

#include "d3q19.hpp"

namespace lbcg {

// Tile loop with an XCD-aware assignment: workgroups are dealt round-robin to
// the 8 XCDs, so the tiles are cut into 8 contiguous chunks and XCD j works
// through chunk j.  Neighbouring tiles (the +-y and +-z stencil partners) then
// share one L2.
struct TileRange { int first, stride, end; };

__device__ inline TileRange tile_range(int ntiles)
{
    const int G = gridDim.x, b = blockIdx.x;
    if (G < 8) return {b, G, ntiles};
    const int j = b & 7, m = b >> 3;
    const int nb = G / 8 + (j < G % 8 ? 1 : 0);
    const int t0 = j * (ntiles / 8) + min(j, ntiles % 8);
    const int t1 = t0 + ntiles / 8 + (j < ntiles % 8 ? 1 : 0);
    return {t0 + m, nb, t1};
}

// Case constants are read-only for the whole launch: reading them through
// the constant address space lets the compiler keep them in scalar registers
// (scalar loads of uniform addresses) instead of per-lane vector registers.
typedef const __attribute__((address_space(4))) DevCase DC;

__device__ inline DC &case_at(const DevCase *cases, int i)
{
    return ((DC *)cases)[i];
}

// Tile entry (case, first node).  The tile index is the same for the whole
// workgroup; reading it through readfirstlane tells the compiler so, which
// keeps the case constants and every buffer base in scalar registers.
__device__ inline int2 uniform_tile(const int2 *tiles, int t)
{
    typedef const __attribute__((address_space(4))) int CI;
    const CI *p = (const CI *)tiles;
    const int tu = __builtin_amdgcn_readfirstlane(t);
    return make_int2(p[2 * tu], p[2 * tu + 1]);
}

struct Coord {
    int x, y, z, node;
    int o[3][3];                 // index offset of the -1, 0, +1 neighbour along x, y, z (periodic wrap)
    bool lo[3], hi[3];           // first / last layer of the wall axis
};

// WL: which walls the cases of the launch may have: WALLS_NONE, WALLS_Z (walls
// only on the z axis, or none) or WALLS_ANY.  With fewer possibilities the
// wall flags of the other axes are compile-time false and the bounce-back and
// ghost-layer code for them folds away.
constexpr int WALLS_NONE = 0, WALLS_Z = 1, WALLS_ANY = 2;

template <int WL = WALLS_ANY>
__device__ inline Coord make_coord(DC &C, int node)
{
    Coord c;
    c.node = node;
    const int nxy = C.nx * C.ny;
    c.z = node / nxy;
    const int r = node - c.z * nxy;
    c.y = r / C.nx;
    c.x = r - c.y * C.nx;
    c.o[0][0] = c.x == 0 ? C.nx - 1 : -1;
    c.o[0][1] = 0;
    c.o[0][2] = c.x == C.nx - 1 ? 1 - C.nx : 1;
    c.o[1][0] = c.y == 0 ? nxy - C.nx : -C.nx;
    c.o[1][1] = 0;
    c.o[1][2] = c.y == C.ny - 1 ? C.nx - nxy : C.nx;
    c.o[2][0] = c.z == 0 ? C.N - nxy : -nxy;
    c.o[2][1] = 0;
    c.o[2][2] = c.z == C.nz - 1 ? nxy - C.N : nxy;
    constexpr bool xy = WL == WALLS_ANY, zz = WL != WALLS_NONE;
    c.lo[0] = xy && C.wall == 0 && c.x == 0; c.hi[0] = xy && C.wall == 0 && c.x == C.nx - 1;
    c.lo[1] = xy && C.wall == 1 && c.y == 0; c.hi[1] = xy && C.wall == 1 && c.y == C.ny - 1;
    c.lo[2] = zz && C.wall == 2 && c.z == 0; c.hi[2] = zz && C.wall == 2 && c.z == C.nz - 1;
    return c;
}

// The same from known coordinates (no division).
template <int WL = WALLS_ANY>
__device__ inline Coord make_coord_xyz(DC &C, int x, int y, int z)
{
    Coord c;
    const int nxy = C.nx * C.ny;
    c.x = x; c.y = y; c.z = z;
    c.node = x + C.nx * y + nxy * z;
    c.o[0][0] = c.x == 0 ? C.nx - 1 : -1;
    c.o[0][1] = 0;
    c.o[0][2] = c.x == C.nx - 1 ? 1 - C.nx : 1;
    c.o[1][0] = c.y == 0 ? nxy - C.nx : -C.nx;
    c.o[1][1] = 0;
    c.o[1][2] = c.y == C.ny - 1 ? C.nx - nxy : C.nx;
    c.o[2][0] = c.z == 0 ? C.N - nxy : -nxy;
    c.o[2][1] = 0;
    c.o[2][2] = c.z == C.nz - 1 ? nxy - C.N : nxy;
    constexpr bool xy = WL == WALLS_ANY, zz = WL != WALLS_NONE;
    c.lo[0] = xy && C.wall == 0 && c.x == 0; c.hi[0] = xy && C.wall == 0 && c.x == C.nx - 1;
    c.lo[1] = xy && C.wall == 1 && c.y == 0; c.hi[1] = xy && C.wall == 1 && c.y == C.ny - 1;
    c.lo[2] = zz && C.wall == 2 && c.z == 0; c.hi[2] = zz && C.wall == 2 && c.z == C.nz - 1;
    return c;
}

// Node at x + (X, Y, Z) with periodic wrap (X, Y, Z in {-1, 0, 1}).
template <int X, int Y, int Z>
__device__ inline int neighbour(const Coord &c)
{
    return c.node + c.o[0][1 + X] + c.o[1][1 + Y] + c.o[2][1 + Z];
}

// Pull source of direction i: the post-collision value at x - e_i, or, when
// x - e_i lies beyond a wall (halfway bounce-back), the opposite direction at
// x itself.
template <int I>
__device__ inline bool bounce(const Coord &c)
{
    constexpr int X = ex(I), Y = ey(I), Z = ez(I);
    return (X == 1 && c.lo[0]) || (X == -1 && c.hi[0]) || (Y == 1 && c.lo[1]) || (Y == -1 && c.hi[1]) ||
           (Z == 1 && c.lo[2]) || (Z == -1 && c.hi[2]);
}

// Wall a bounce-back of direction i reflects at: 0 low, 1 high, -1 none.
template <int I>
__device__ inline int bounce_side(const Coord &c)
{
    constexpr int X = ex(I), Y = ey(I), Z = ez(I);
    const bool lo = (X == 1 && c.lo[0]) || (Y == 1 && c.lo[1]) || (Z == 1 && c.lo[2]);
    const bool hi = (X == -1 && c.hi[0]) || (Y == -1 && c.hi[1]) || (Z == -1 && c.hi[2]);
    return lo ? 0 : (hi ? 1 : -1);
}

// e_i . U_w of the wall a bounce-back of direction i reflects at.  A
// reflected population of colour k gains wg[k][class] * rho_k * (e_i . U_w):
// twice the odd part of the equilibrium at the wall velocity, so that a
// uniform flow at U_w is left unchanged by the wall.
template <int I>
__device__ inline float wall_eu(DC &C, int side)
{
    return ex(I) * C.uw[side][0] + ey(I) * C.uw[side][1] + ez(I) * C.uw[side][2];
}

template <int I>
__device__ inline void pull_source(DC &, const Coord &c, int &src, int &dir)
{
    const bool bb = bounce<I>(c);
    src = bb ? c.node : neighbour<-ex(I), -ey(I), -ez(I)>(c);
    dir = bb ? opp(I) : I;
}

struct NodeState {
    float h[Q];                  // sum_k (rho_k(src) - S_k) phi_i^k + d_i^k
    float R[2];                  // colour densities R_k = fl(S_k + eps_k)
    float D[2];                  // R_k - S_k (exact)
    float eta[2];                // eps_k - (R_k - S_k): what R_k could not hold
    float jx, jy, jz;            // sum_i e_i f_i (the rest state carries none)
};

// Direction i and its opposite are stored next to each other ((1,2), (3,4),
// ..., (17,18); 0 alone), so one buffer resource spans both and a bounce-back
// lane differs from its neighbours only in the offset it supplies.
template <int I>
constexpr int pair_first() { return I == 0 ? 0 : ((I & 1) ? I : I - 1); }

// MV: the launch holds a case with a moving wall (a separate instantiation, so
// that cases at rest pay nothing for the wall-gain code).
template <int ST, bool MV, int CPP, int I>
__device__ inline void pull_one(const StepArgs &a, DC &C, const Coord &c, const float2 own,
                                NodeState &s, float &eR, float &eB)
{
    using S = Storage<ST>;
    using P = typename S::P;
    constexpr int F = pair_first<I>(), W = I == 0 ? 1 : 2;
    const size_t N = (size_t)C.N, NS = (size_t)C.NS;
    const P *base = reinterpret_cast<const P *>(a.fin) + C.pop_off / 2;
    const bool bb = bounce<I>(c);
    const uint32_t si = (uint32_t)(bb ? c.node : neighbour<-ex(I), -ey(I), -ez(I)>(c));
    constexpr bool hi_own = I != F, hi_opp = opp(I) != F;          // second array of the pair?
    const bool hi = bb ? hi_opp : hi_own;
    const uint32_t e = si + (hi ? (uint32_t)NS : 0u);
    const P v = buf_ld<P, CPP>(rsrc(base + (size_t)F * NS, W * NS * sizeof(P)), e * (uint32_t)sizeof(P));
    const float dR = S::dec(v.r, a.inv_scale);
    const float dB = S::dec(v.b, a.inv_scale);
    const float2 ps = buf_ld<float2, CP_DEFAULT>(rsrc(a.rho_prev + C.node_off, N * sizeof(float2)), si * 8u);
    float tR = __builtin_fmaf(ps.x - own.x, C.phi[0][ecls(I)], dR);
    float tB = __builtin_fmaf(ps.y - own.y, C.phi[1][ecls(I)], dB);
    if constexpr (MV && I != 0) {
        if (C.moving && bb) {        // moving wall: the reflected population gains its momentum
            const float eu = wall_eu<I>(C, bounce_side<I>(c));
            tR = __builtin_fmaf(eu * C.wg[0][ecls(I) - 1], own.x, tR);
            tB = __builtin_fmaf(eu * C.wg[1][ecls(I) - 1], own.y, tB);
        }
    }
    const float h = tR + tB;
    s.h[I] = h;
    eR += tR;
    eB += tB;
    if constexpr (ex(I) == 1) s.jx += h;
    if constexpr (ex(I) == -1) s.jx -= h;
    if constexpr (ey(I) == 1) s.jy += h;
    if constexpr (ey(I) == -1) s.jy -= h;
    if constexpr (ez(I) == 1) s.jz += h;
    if constexpr (ez(I) == -1) s.jz -= h;
}

template <int ST, bool MV, int CPP, int I = 0>
__device__ inline void pull_all(const StepArgs &a, DC &C, const Coord &c, const float2 own,
                                NodeState &s, float &eR, float &eB)
{
    if constexpr (I < Q) {
        pull_one<ST, MV, CPP, I>(a, C, c, own, s, eR, eB);
        pull_all<ST, MV, CPP, I + 1>(a, C, c, own, s, eR, eB);
    }
}

// The same pull with the writers' densities read from an LDS copy of the
// stored-density planes z-1, z, z+1 (rl[0..2], row length RW; ri: the node's
// index in a plane) instead of from memory.  A bounce-back lane takes its own
// density (its slot read is discarded), as the memory form does.
// Fused tiles are FTX x FTY columns: 32 x 8, so that a tile row of 4-byte
// values fills one 128-byte cache line (a wave's load touches 2 lines, where
// 16 x 16 tiles touched 4 half lines) and only 2 x 8 of the halo lies in
// strided columns.
constexpr int FTX = 32, FTY = 8;
constexpr int FNT = FTX * FTY, FNW = FNT / 64;   // lanes and waves of a fused workgroup
static_assert((FNW & (FNW - 1)) == 0, "the halo duty rotates over a power-of-two number of waves");
constexpr int RH = 2;                    // halo of the stored-density planes around a fused tile
constexpr int RW = FTX + 2 * RH, RREG = RW * (FTY + 2 * RH);

// Issue phase: the 19 population loads of a node, all in flight at once.
// SO: the case's level (19 NS pairs) lies below 2^31 bytes and is read
// through one buffer resource, each direction pair's arrays reached by a
// scalar offset; otherwise each pair has a resource of its own.
template <int ST, int CPP, bool SO = false, int I = 0>
__device__ inline void pull_issue(const StepArgs &a, DC &C, const Coord &c, typename Storage<ST>::P (&v)[Q])
{
    if constexpr (I < Q) {
        using P = typename Storage<ST>::P;
        constexpr int F = pair_first<I>(), W = I == 0 ? 1 : 2;
        const size_t NS = (size_t)C.NS;
        const P *base = reinterpret_cast<const P *>(a.fin) + C.pop_off / 2;
        const bool bb = bounce<I>(c);
        const uint32_t si = (uint32_t)(bb ? c.node : neighbour<-ex(I), -ey(I), -ez(I)>(c));
        constexpr bool hi_own = I != F, hi_opp = opp(I) != F;
        const bool hi = bb ? hi_opp : hi_own;
        const uint32_t e = si + (hi ? (uint32_t)NS : 0u);
        if constexpr (SO)
            v[I] = buf_ld_so<P, CPP>(rsrc(base, 19 * NS * sizeof(P)), e * (uint32_t)sizeof(P),
                                     (uint32_t)(F * NS * sizeof(P)));
        else
            v[I] = buf_ld<P, CPP>(rsrc(base + (size_t)F * NS, W * NS * sizeof(P)), e * (uint32_t)sizeof(P));
        pull_issue<ST, CPP, SO, I + 1>(a, C, c, v);
    }
}

// Decode phase: deviations plus the writers' densities from the LDS plane
// ring (as pull_one does with the densities from memory).
template <int ST, bool MV, int I = 0>
__device__ inline void pull_decode(const StepArgs &a, DC &C, const Coord &c, const float2 own,
                                   const float2 *const (&rl)[3], int ri, const typename Storage<ST>::P (&v)[Q],
                                   NodeState &s, float &eR, float &eB)
{
    if constexpr (I < Q) {
        using S = Storage<ST>;
        const bool bb = bounce<I>(c);
        const float dR = S::dec(v[I].r, a.inv_scale);
        const float dB = S::dec(v[I].b, a.inv_scale);
        const float2 pl = rl[1 - ez(I)][ri - ex(I) - RW * ey(I)];
        const float2 ps = bb ? own : pl;
        float tR = __builtin_fmaf(ps.x - own.x, C.phi[0][ecls(I)], dR);
        float tB = __builtin_fmaf(ps.y - own.y, C.phi[1][ecls(I)], dB);
        if constexpr (MV && I != 0) {
            if (C.moving && bb) {
                const float eu = wall_eu<I>(C, bounce_side<I>(c));
                tR = __builtin_fmaf(eu * C.wg[0][ecls(I) - 1], own.x, tR);
                tB = __builtin_fmaf(eu * C.wg[1][ecls(I) - 1], own.y, tB);
            }
        }
        const float h = tR + tB;
        s.h[I] = h;
        eR += tR;
        eB += tB;
        if constexpr (ex(I) == 1) s.jx += h;
        if constexpr (ex(I) == -1) s.jx -= h;
        if constexpr (ey(I) == 1) s.jy += h;
        if constexpr (ey(I) == -1) s.jy -= h;
        if constexpr (ez(I) == 1) s.jz += h;
        if constexpr (ez(I) == -1) s.jz -= h;
        pull_decode<ST, MV, I + 1>(a, C, c, own, rl, ri, v, s, eR, eB);
    }
}

// The node state from the loaded populations of node c (ri: its index in
// the density planes).
template <int ST, bool MV>
__device__ inline void pull_finish(const StepArgs &a, DC &C, const Coord &c, const float2 *const (&rl)[3], int ri,
                                   const typename Storage<ST>::P (&v)[Q], NodeState &s)
{
    const float2 own = rl[1][ri];
    float eR = 0.f, eB = 0.f;
    s.jx = s.jy = s.jz = 0.f;
    pull_decode<ST, MV>(a, C, c, own, rl, ri, v, s, eR, eB);
    s.R[0] = own.x + eR;
    s.R[1] = own.y + eB;
    s.D[0] = s.R[0] - own.x;
    s.D[1] = s.R[1] - own.y;
    s.eta[0] = eR - s.D[0];
    s.eta[1] = eB - s.D[1];
}

// ------------------------------------------------------ compact levels
// A compact level (LV_COMPACT in d3q19.hpp): direction 0 is the writer's own
// (red, blue) pair at pair index node; direction i >= 1 is one total
// deviation at element (i + 1) NS + node, so i and its opposite are again
// adjacent arrays.  A puller rebuilds the red share of each value from the
// writer's data (rho_R, rho_B; rho_R/rho, g; cr) exactly as the writer's
// recoloring defines it, and the blue share as the rest of the total.

// e_i . (d.y, d.z, d.w)
template <int I>
__device__ inline float e_dot(const float4 &d)
{
    constexpr int X = ex(I), Y = ey(I), Z = ez(I);
    if constexpr (X != 0 && Y != 0) return X * d.y + Y * d.z;
    else if constexpr (X != 0 && Z != 0) return X * d.y + Z * d.w;
    else if constexpr (Y != 0 && Z != 0) return Y * d.z + Z * d.w;
    else if constexpr (X != 0) return X * d.y;
    else if constexpr (Y != 0) return Y * d.z;
    else return Z * d.w;
}

// One pulled value t of direction I >= 1 with its writer's data (rw: rho_R,
// rho_B; dw: rho_R/rho, g; cw: axis-class cr).  bb: the value is the node's
// own opposite direction (halfway bounce-back), whose segregation term has
// the opposite sign.
template <int ST, bool MV, int I>
__device__ inline void decode_c(DC &C, const Coord &c, const float2 own, bool bb, float t, float2 rw, float4 dw,
                                float cw, NodeState &s, float &eR, float &eB)
{
    constexpr int cl = ecls(I);
    const float eg = e_dot<I>(dw);
    float seg = cl == 1 ? eg : kDiagSeg * eg;
    if (bb) seg = -seg;
    const float crc = cl == 1 ? cw : 0.5f * cw;
    const float dR = __builtin_fmaf(dw.x, t, seg + crc);
    float tR = __builtin_fmaf(rw.x - own.x, C.phi[0][cl], dR);
    float tB = __builtin_fmaf(rw.y - own.y, C.phi[1][cl], t - dR);
    if constexpr (MV) {
        if (C.moving && bb) {        // moving wall: the reflected population gains its momentum
            const float eu = wall_eu<I>(C, bounce_side<I>(c));
            tR = __builtin_fmaf(eu * C.wg[0][cl - 1], own.x, tR);
            tB = __builtin_fmaf(eu * C.wg[1][cl - 1], own.y, tB);
        }
    }
    const float h = tR + tB;
    s.h[I] = h;
    eR += tR;
    eB += tB;
    if constexpr (ex(I) == 1) s.jx += h;
    if constexpr (ex(I) == -1) s.jx -= h;
    if constexpr (ey(I) == 1) s.jy += h;
    if constexpr (ey(I) == -1) s.jy -= h;
    if constexpr (ez(I) == 1) s.jz += h;
    if constexpr (ez(I) == -1) s.jz -= h;
}

// Loaded values of one compact pull: the own pair of direction 0 and the
// totals of directions 1-18 (v[0] unused).
template <int ST> struct CompactPull {
    typename Storage<ST>::P v0;
    typename Storage<ST>::T v[Q];
};

// SO: the case's whole level lies within one buffer resource (20 NS values
// below 2^31 bytes), and each direction pair's array is reached by a scalar
// offset; otherwise each pair has a resource of its own (any size, but the
// ten resources stay live in scalar registers across the plane loop).
template <int ST, int CPP, bool SO = false, int I = 1>
__device__ inline void pull_issue_c(const StepArgs &a, DC &C, const Coord &c, CompactPull<ST> &p)
{
    using S = Storage<ST>;
    using T = typename S::T;
    using P = typename S::P;
    const size_t NS = (size_t)C.NS;
    const T *base0 = reinterpret_cast<const T *>(a.fin) + C.pop_off;
    if constexpr (I == 1) {
        if constexpr (SO)
            p.v0 = buf_ld_so<P, CPP>(rsrc(base0, 20 * NS * sizeof(T)), (uint32_t)c.node * (uint32_t)sizeof(P), 0u);
        else
            p.v0 = buf_ld<P, CPP>(rsrc(base0, NS * sizeof(P)), (uint32_t)c.node * (uint32_t)sizeof(P));
    }
    if constexpr (I < Q) {
        constexpr int F = pair_first<I>();
        const bool bb = bounce<I>(c);
        const uint32_t si = (uint32_t)(bb ? c.node : neighbour<-ex(I), -ey(I), -ez(I)>(c));
        constexpr bool hi_own = I != F, hi_opp = opp(I) != F;
        const bool hi = bb ? hi_opp : hi_own;
        const uint32_t e = si + (hi ? (uint32_t)NS : 0u);
        if constexpr (SO)
            p.v[I] = buf_ld_so<T, CPP>(rsrc(base0, 20 * NS * sizeof(T)), e * (uint32_t)sizeof(T),
                                       (uint32_t)((F + 1) * NS * sizeof(T)));
        else
            p.v[I] = buf_ld<T, CPP>(rsrc(base0 + (size_t)(F + 1) * NS, 2 * NS * sizeof(T)), e * (uint32_t)sizeof(T));
        pull_issue_c<ST, CPP, SO, I + 1>(a, C, c, p);
    }
}

// LDS rings of the writers' data of planes z-1, z, z+1 (as the density ring).
struct WriterRing {
    const float2 *r[3];
    const float4 *d[3];
    const float *c[3];
};

template <int ST, bool MV, int I = 1>
__device__ inline void pull_decode_c(const StepArgs &a, DC &C, const Coord &c, const float2 own,
                                     const WriterRing &wr, int ri, const CompactPull<ST> &p, NodeState &s,
                                     float &eR, float &eB)
{
    if constexpr (I < Q) {
        using S = Storage<ST>;
        const bool bb = bounce<I>(c);
        const int li = bb ? ri : ri - ex(I) - RW * ey(I);
        const float2 *R = bb ? wr.r[1] : wr.r[1 - ez(I)];
        const float4 *D = bb ? wr.d[1] : wr.d[1 - ez(I)];
        const float *Cw = bb ? wr.c[1] : wr.c[1 - ez(I)];
        decode_c<ST, MV, I>(C, c, own, bb, S::dec(p.v[I], a.inv_scale), R[li], D[li], Cw[li], s, eR, eB);
        pull_decode_c<ST, MV, I + 1>(a, C, c, own, wr, ri, p, s, eR, eB);
    }
}

template <int ST>
__device__ inline void own_pair(const StepArgs &a, const typename Storage<ST>::P &v0, NodeState &s, float &eR,
                                float &eB)
{
    using S = Storage<ST>;
    const float dR = S::dec(v0.r, a.inv_scale), dB = S::dec(v0.b, a.inv_scale);
    s.h[0] = dR + dB;
    eR = dR;
    eB = dB;
}

__device__ inline void finish_state(const float2 own, float eR, float eB, NodeState &s)
{
    s.R[0] = own.x + eR;
    s.R[1] = own.y + eB;
    s.D[0] = s.R[0] - own.x;
    s.D[1] = s.R[1] - own.y;
    s.eta[0] = eR - s.D[0];
    s.eta[1] = eB - s.D[1];
}

// The node state from a compact pull, writers' data from the LDS rings.
template <int ST, bool MV>
__device__ inline void pull_finish_c(const StepArgs &a, DC &C, const Coord &c, const WriterRing &wr, int ri,
                                     const CompactPull<ST> &p, NodeState &s)
{
    const float2 own = wr.r[1][ri];
    float eR, eB;
    s.jx = s.jy = s.jz = 0.f;
    own_pair<ST>(a, p.v0, s, eR, eB);
    pull_decode_c<ST, MV>(a, C, c, own, wr, ri, p, s, eR, eB);
    finish_state(own, eR, eB, s);
}

// The same with the writers' data read from memory (diagnostics).
template <int ST, bool MV, int I = 1>
__device__ inline void pull_mem_c(const StepArgs &a, DC &C, const Coord &c, const float2 own,
                                  const CompactPull<ST> &p, NodeState &s, float &eR, float &eB)
{
    if constexpr (I < Q) {
        using S = Storage<ST>;
        const bool bb = bounce<I>(c);
        const int si = bb ? c.node : neighbour<-ex(I), -ey(I), -ez(I)>(c);
        const size_t o = (size_t)C.node_off + si;
        decode_c<ST, MV, I>(C, c, own, bb, S::dec(p.v[I], a.inv_scale), a.rho_prev[o], a.dsc_prev[o],
                            a.crs_prev[o], s, eR, eB);
        pull_mem_c<ST, MV, I + 1>(a, C, c, own, p, s, eR, eB);
    }
}

template <int ST, bool MV>
__device__ inline void pull_node_c(const StepArgs &a, DC &C, const Coord &c, NodeState &s)
{
    CompactPull<ST> p;
    pull_issue_c<ST, CP_DEFAULT>(a, C, c, p);
    const float2 own = a.rho_prev[C.node_off + c.node];
    float eR, eB;
    s.jx = s.jy = s.jz = 0.f;
    own_pair<ST>(a, p.v0, s, eR, eB);
    pull_mem_c<ST, MV>(a, C, c, own, p, s, eR, eB);
    finish_state(own, eR, eB, s);
}

// CPP: cache policy of the population loads (streaming unless the same
// populations are read again soon).
template <int ST, bool MV, int CPP = CP_STREAM>
__device__ inline void pull_node(const StepArgs &a, DC &C, const Coord &c, NodeState &s)
{
    const float2 own = buf_ld<float2, CP_DEFAULT>(rsrc(a.rho_prev + C.node_off, (size_t)C.N * sizeof(float2)),
                                                  (uint32_t)c.node * 8u);
    float eR = 0.f, eB = 0.f;
    s.jx = s.jy = s.jz = 0.f;
    pull_all<ST, MV, CPP>(a, C, c, own, s, eR, eB);
    s.R[0] = own.x + eR;
    s.R[1] = own.y + eB;
    s.D[0] = s.R[0] - own.x;
    s.D[1] = s.R[1] - own.y;
    s.eta[0] = eR - s.D[0];
    s.eta[1] = eB - s.D[1];
}

// Force density (reading: uniform part plus buoyancy) and u = (j + F/2)/rho.
struct Macro { float rho, inv_rho, Fx, Fy, Fz, ux, uy, uz; };

__device__ inline Macro macro(DC &C, const NodeState &s)
{
    Macro m;
    m.rho = s.R[0] + s.R[1];
    // hardware reciprocal (1 ulp): 1/rho scales u only; rho_R/rho of the
    // recoloring and the phase field keep correctly rounded quotients
    m.inv_rho = __builtin_amdgcn_rcpf(m.rho);
    const float dr = m.rho - C.rho_ref;
    m.Fx = C.F[0] + dr * C.g[0];
    m.Fy = C.F[1] + dr * C.g[1];
    m.Fz = C.F[2] + dr * C.g[2];
    m.ux = (s.jx + 0.5f * m.Fx) * m.inv_rho;
    m.uy = (s.jy + 0.5f * m.Fy) * m.inv_rho;
    m.uz = (s.jz + 0.5f * m.Fz) * m.inv_rho;
    return m;
}

__device__ inline float phase_field(DC &C, float rR, float rB)
{
    const float a = rR * C.rin_inv[0], b = rB * C.rin_inv[1];
    return (a - b) / (a + b);
}

// ----------------------------------------------------------------- k_aux
template <int ST, bool MV, int WL>
__global__ __launch_bounds__(256) void k_aux(StepArgs a)
{
    const TileRange tr = tile_range(a.ntiles);
    for (int t = tr.first; t < tr.end; t += tr.stride) {
        const int2 tl = uniform_tile(a.tiles, t);
        DC &C = case_at(a.cases, tl.x);
        const int node = tl.y + (int)threadIdx.x;
        if (node >= C.N) continue;
        const Coord c = make_coord<WL>(C, node);
        NodeState s;
        pull_node<ST, MV>(a, C, c, s);
        const Macro m = macro(C, s);
        const float qs = s.R[0] * C.qc[0] + s.R[1] * C.qc[1];
        a.aux[C.node_off + node] = make_float4(phase_field(C, s.R[0], s.R[1]), m.ux * qs, m.uy * qs, m.uz * qs);
        if (MV && C.moving && (c.lo[C.wall] || c.hi[C.wall])) {
            // first-layer density factor of Qbar for the ghost layer of a moving wall
            const int w = C.wall, b = w == 0 ? 1 : 0, cax = w == 2 ? 1 : 2;
            const int co[3] = {c.x, c.y, c.z};
            const int n[3] = {C.nx, C.ny, C.nz};
            const int pi = co[b] + n[b] * co[cax];
            if (c.lo[w]) a.wallq[C.ghost_off + pi] = qs;
            if (c.hi[w]) a.wallq[C.ghost_off + C.plane + pi] = qs;
        }
    }
}

// --------------------------------------------------------------- k_ghost
// One entry per wall-plane node and side.  The ghost phase field follows the
// geometric wetting rule: across the half link to the ghost, rho^N changes by
// cot(theta) |grad_par rho^N| (2D isotropic stencil on the first layer), so
// that the interface meets the wall at theta through the red fluid.  Qbar,
// which carries u (zero on the halfway wall), is reflected oddly.
__global__ __launch_bounds__(256) void k_ghost(StepArgs a, const int2 *gtiles, int ngtiles)
{
    for (int t = blockIdx.x; t < ngtiles; t += gridDim.x) {
        const int2 tl = gtiles[t];
        DC &C = case_at(a.cases, tl.x);
        const int e = tl.y + (int)threadIdx.x;
        if (e >= 2 * C.plane) continue;
        const int side = e >= C.plane ? 1 : 0;
        const int pi = e - side * C.plane;
        int n[3] = {C.nx, C.ny, C.nz};
        const int w = C.wall, b = w == 0 ? 1 : 0, cax = w == 2 ? 1 : 2;
        const int ib = pi % n[b], ic = pi / n[b];
        int q[3];
        q[w] = side ? n[w] - 1 : 0;
        float gb = 0.f, gc = 0.f;
        #pragma unroll
        for (int db = -1; db <= 1; ++db) {
            #pragma unroll
            for (int dc = -1; dc <= 1; ++dc) {
                if (db == 0 && dc == 0) continue;
                const float wgt = (db != 0 && dc != 0) ? (1.0f / 12.0f) : (1.0f / 3.0f);
                int vb = ib + db, vc = ic + dc;
                vb = vb < 0 ? n[b] - 1 : (vb >= n[b] ? 0 : vb);
                vc = vc < 0 ? n[cax] - 1 : (vc >= n[cax] ? 0 : vc);
                q[b] = vb; q[cax] = vc;
                const float v = a.aux[C.node_off + q[0] + C.nx * (q[1] + C.ny * q[2])].x;
                gb += wgt * (float)db * v;
                gc += wgt * (float)dc * v;
            }
        }
        q[b] = ib; q[cax] = ic;
        const float4 s = a.aux[C.node_off + q[0] + C.nx * (q[1] + C.ny * q[2])];
        const float gpar = sqrtf(gb * gb + gc * gc);
        // Qbar takes the wall's value half way: ghost = 2 Qbar(wall) - Qbar(first
        // layer), Qbar(wall) = U_w sum_k rho_k (1 - 3 c_s^k^2) of the first layer
        const float qw = C.moving ? 2.0f * a.wallq[C.ghost_off + e] : 0.f;
        a.ghost[C.ghost_off + e] = make_float4(s.x + C.cot[side] * gpar, qw * C.uw[side][0] - s.y,
                                               qw * C.uw[side][1] - s.z, qw * C.uw[side][2] - s.w);
    }
}

// Aux value at x + e (or the ghost beyond a wall).  The aux read is issued
// for every lane (a ghost lane reads its own node) so that no buffer access
// sits in divergent control flow.
template <int X, int Y, int Z>
__device__ inline float4 aux_at(const StepArgs &a, DC &C, const Coord &c)
{
    const bool glo = (X == -1 && c.lo[0]) || (Y == -1 && c.lo[1]) || (Z == -1 && c.lo[2]);
    const bool ghi = (X == 1 && c.hi[0]) || (Y == 1 && c.hi[1]) || (Z == 1 && c.hi[2]);
    const uint32_t nb = (uint32_t)(glo || ghi ? c.node : neighbour<X, Y, Z>(c));
    float4 v = buf_ld<float4, CP_DEFAULT>(rsrc(a.aux + C.node_off, (size_t)C.N * sizeof(float4)), nb * 16u);
    if (glo || ghi) {
        // wrapped coordinates of x + e within the wall plane
        const int px = c.x + X < 0 ? C.nx - 1 : (c.x + X >= C.nx ? 0 : c.x + X);
        const int py = c.y + Y < 0 ? C.ny - 1 : (c.y + Y >= C.ny ? 0 : c.y + Y);
        const int pz = c.z + Z < 0 ? C.nz - 1 : (c.z + Z >= C.nz ? 0 : c.z + Z);
        const int gi = C.wall == 0 ? py + C.ny * pz : (C.wall == 1 ? px + C.nx * pz : px + C.nx * py);
        v = a.ghost[C.ghost_off + (ghi ? C.plane : 0) + gi];
    }
    return v;
}

// Eq. (49) for rho^N (all components) and for Qbar_alpha (component alpha only).
struct Stencil { float gx, gy, gz, Qx, Qy, Qz; };

template <int I = 1>
__device__ inline void stencil_acc(const StepArgs &a, DC &C, const Coord &c, Stencil &st)
{
    if constexpr (I < Q) {
        constexpr int X = ex(I), Y = ey(I), Z = ez(I);
        constexpr float w3 = ecls(I) == 1 ? (1.0f / 6.0f) : (1.0f / 12.0f);   // 3 w_i
        const float4 v = aux_at<X, Y, Z>(a, C, c);
        if constexpr (X != 0) { st.gx += (X * w3) * v.x; st.Qx += (X * w3) * v.y; }
        if constexpr (Y != 0) { st.gy += (Y * w3) * v.x; st.Qy += (Y * w3) * v.z; }
        if constexpr (Z != 0) { st.gz += (Z * w3) * v.x; st.Qz += (Z * w3) * v.w; }
        stencil_acc<I + 1>(a, C, c, st);
    }
}

// Eq. (52) with the quadratic joins (reading: harmonic mean at rho^N = 0,
// zero slope where they meet tau_v^R / tau_v^B at +-delta).
__device__ inline float tau_v(DC &C, float rn)
{
    if (rn > C.delta) return C.tauR;
    if (rn < -C.delta) return C.tauB;
    if (rn > 0.f) return C.s1 + rn * (C.s2 + rn * C.s3);
    return C.s1 + rn * (C.t2 + rn * C.t3);
}

// ------------------------------------------------------------- collision
// One node: tau_v (Eq. 52), the two-colour MRT collision in moment space with
// correction term, body force and perturbation (Eq. 41-45, 53), recoloring
// (Eq. 10-11) and the store of both colours' deviations at the node's own
// slots.  st: colour gradient and Q_alpha (Eq. 49); rn: the node's rho^N.
// OUT: level format written (LV_PAIR, or LV_COMPACT: the total deviations
// plus the writer's recoloring data, from which the pullers rebuild the red
// shares this function would have stored).
template <int ST, int CPS = CP_DEFAULT, int OUT = LV_PAIR>
__device__ inline void collide_node(const StepArgs &a, DC &C, int node, const NodeState &s,
                                    const Stencil &st, float rn)
{
    using S = Storage<ST>;
    using T = typename S::T;
    const Macro M = macro(C, s);
    const float ux = M.ux, uy = M.uy, uz = M.uz, rho = M.rho;

    const float tv = tau_v(C, rn);
    const float sv = __builtin_amdgcn_rcpf(tv), se = C.s_e, sq = C.s_q, sp = C.s_pi;   // 1/tau_v to 1 ulp

    // g_i = f_i - sum_k R_k phi_i^k, per velocity class
    const float dc0 = s.D[0] * C.phi[0][0] + s.D[1] * C.phi[1][0];
    const float dc1 = s.D[0] * C.phi[0][1] + s.D[1] * C.phi[1][1];
    const float dc2 = s.D[0] * C.phi[0][2] + s.D[1] * C.phi[1][2];
    float f[Q];
    f[0] = s.h[0] - dc0;
    #pragma unroll
    for (int i = 1; i < 7; ++i) f[i] = s.h[i] - dc1;
    #pragma unroll
    for (int i = 7; i < Q; ++i) f[i] = s.h[i] - dc2;
    // raw moments M g (Eq. 43, Appendix), rows 4-18; the rest state adds
    // 3p_R to row 4 and p_R/3 to rows 16-18 (p_R = sum_k R_k (c_s^k)^2)
    const float d78 = f[7] + f[8], d910 = f[9] + f[10];
    const float d1112 = f[11] + f[12], d1314 = f[13] + f[14];
    const float d1516 = f[15] + f[16], d1718 = f[17] + f[18];
    const float a12 = f[1] + f[2], a34 = f[3] + f[4], a56 = f[5] + f[6];
    const float m16 = d78 + d910, m17 = d1112 + d1314, m18 = d1516 + d1718;
    const float m4 = a12 + a34 + a56 + 2.0f * (m16 + m17 + m18);
    const float m5 = 2.0f * a12 - a34 - a56 + m16 + m17 - 2.0f * m18;
    const float m6 = a34 - a56 + m16 - m17;
    const float m7 = d78 - d910, m8 = d1112 - d1314, m9 = d1516 - d1718;
    const float m10 = f[7] - f[8] - f[9] + f[10];
    const float m11 = f[7] - f[8] + f[9] - f[10];
    const float m12 = f[11] - f[12] - f[13] + f[14];
    const float m13 = f[11] - f[12] + f[13] - f[14];
    const float m14 = f[15] - f[16] - f[17] + f[18];
    const float m15 = f[15] - f[16] + f[17] - f[18];

    // two-colour equilibria sum_k m^{k,eq} (Appendix rows 0-15; rows
    // 16-18 as M f^eq, or as the Appendix prints them) minus the rest-state
    // moments; p = sum_k rho_k (c_s^k)^2
    const float p = s.R[0] * C.cs2[0] + s.R[1] * C.cs2[1];
    const float pe = s.eta[0] * C.cs2[0] + s.eta[1] * C.cs2[1];
    const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz, uu = uxx + uyy + uzz;
    const float e4 = 3.0f * pe + rho * uu;
    const float e5 = rho * (2.0f * uxx - uyy - uzz);
    const float e6 = rho * (uyy - uzz);
    const float e7 = rho * ux * uy, e8 = rho * ux * uz, e9 = rho * uy * uz;
    const float p3 = C.improved ? p : rho * (1.0f / 3.0f);
    const float e10 = p3 * uy, e11 = p3 * ux, e12 = p3 * uz;
    const float e16b = (2.0f * pe - rho * uu) * (1.0f / 6.0f);
    const float rc16 = C.c16 * rho;
    const float e16 = e16b + rc16 * (uxx + uyy);
    const float e17 = e16b + rc16 * (uxx + uzz);
    const float e18 = e16b + rc16 * (uyy + uzz);

    // correction term (Eq. 45), summed over the colours
    float c4 = 0.f, c5 = 0.f, c6 = 0.f;
    if (C.improved) {
        c4 = st.Qx + st.Qy + st.Qz;
        c5 = 2.0f * st.Qx - st.Qy - st.Qz;
        c6 = st.Qy - st.Qz;
    }
    // body force in moment space (reading: Guo's source, M F^Guo)
    const float Fx = M.Fx, Fy = M.Fy, Fz = M.Fz;
    const float uFx = ux * Fx, uFy = uy * Fy, uFz = uz * Fz;
    const float f4 = 2.0f * (uFx + uFy + uFz);
    const float f5 = 2.0f * (2.0f * uFx - uFy - uFz);
    const float f6 = 2.0f * (uFy - uFz);
    const float f7 = ux * Fy + uy * Fx, f8 = ux * Fz + uz * Fx, f9 = uy * Fz + uz * Fy;
    const float t3 = 1.0f / 3.0f;
    const float f16 = (2.0f * uFx + 2.0f * uFy - uFz) * t3;
    const float f17 = (2.0f * uFx - uFy + 2.0f * uFz) * t3;
    const float f18 = (-uFx + 2.0f * uFy + 2.0f * uFz) * t3;
    // perturbation in moment space: M Omega2 summed over the colours
    // (Eq. 8), relaxed by S (Eq. 53)
    const float g2 = st.gx * st.gx + st.gy * st.gy + st.gz * st.gz;
    float o4 = 0.f, o5 = 0.f, o6 = 0.f, o7 = 0.f, o8 = 0.f, o9 = 0.f, o16 = 0.f, o17 = 0.f, o18 = 0.f;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (g2 > 1e-24f) {
        const float ig = rsqrtf(g2);
        nx = st.gx * ig; ny = st.gy * ig; nz = st.gz * ig;
        const float ag = C.Asum * ig * (1.0f / 9.0f);
        const float gxx = st.gx * st.gx, gyy = st.gy * st.gy, gzz = st.gz * st.gz;
        o4 = -2.0f * ag * g2;
        o5 = ag * (3.0f * gxx - g2);
        o6 = ag * (gyy - gzz);
        o7 = ag * st.gx * st.gy; o8 = ag * st.gx * st.gz; o9 = ag * st.gy * st.gz;
        o16 = -0.5f * ag * gzz; o17 = -0.5f * ag * gyy; o18 = -0.5f * ag * gxx;
    }
    // post-collision moment changes mbar (Eq. 41 + force + Eq. 53); rows
    // 0-3: mass unchanged, momentum changed by F (exact for the sum)
    const float he = 1.0f - 0.5f * se, hv = 1.0f - 0.5f * sv, hq = 1.0f - 0.5f * sq, hp = 1.0f - 0.5f * sp;
    const float b4 = -se * (m4 - e4) + he * (c4 + f4) + se * o4;
    const float b5 = -sv * (m5 - e5) + hv * (c5 + f5) + sv * o5;
    const float b6 = -sv * (m6 - e6) + hv * (c6 + f6) + sv * o6;
    const float b7 = -sv * (m7 - e7) + hv * f7 + sv * o7;
    const float b8 = -sv * (m8 - e8) + hv * f8 + sv * o8;
    const float b9 = -sv * (m9 - e9) + hv * f9 + sv * o9;
    const float b10 = -sq * (m10 - e10) + hq * (Fy * t3);
    const float b11 = -sq * (m11 - e11) + hq * (Fx * t3);
    const float b12 = -sq * (m12 - e12) + hq * (Fz * t3);
    const float b13 = -sq * (m13 - e11) + hq * (Fx * t3);
    const float b14 = -sq * (m14 - e12) + hq * (Fz * t3);
    const float b15 = -sq * (m15 - e10) + hq * (Fy * t3);
    const float b16 = -sp * (m16 - e16) + hp * f16 + sp * o16;
    const float b17 = -sp * (m17 - e17) + hp * f17 + sp * o17;
    const float b18 = -sp * (m18 - e18) + hp * f18 + sp * o18;

    // t = g + M^-1 mbar = f* - sum_k R_k phi^k (sparse closed form of M^-1)
    float fs[Q];
    const float q4 = b4 * (1.0f / 6.0f);
    fs[0] = f[0] - b4 + b16 + b17 + b18;
    {
        const float base = q4 + b5 * (1.0f / 6.0f) - 0.5f * (b16 + b17);
        const float odd = 0.5f * (Fx - b11 - b13);
        fs[1] = f[1] + base + odd;
        fs[2] = f[2] + base - odd;
    }
    {
        const float base = q4 - b5 * (1.0f / 12.0f) + 0.25f * b6 - 0.5f * (b16 + b18);
        const float odd = 0.5f * (Fy - b10 - b15);
        fs[3] = f[3] + base + odd;
        fs[4] = f[4] + base - odd;
    }
    {
        const float base = q4 - b5 * (1.0f / 12.0f) - 0.25f * b6 - 0.5f * (b17 + b18);
        const float odd = 0.5f * (Fz - b12 - b14);
        fs[5] = f[5] + base + odd;
        fs[6] = f[6] + base - odd;
    }
    fs[7] = f[7] + 0.25f * (b7 + b10 + b11 + b16);
    fs[8] = f[8] + 0.25f * (b7 - b10 - b11 + b16);
    fs[9] = f[9] + 0.25f * (-b7 - b10 + b11 + b16);
    fs[10] = f[10] + 0.25f * (-b7 + b10 - b11 + b16);
    fs[11] = f[11] + 0.25f * (b8 + b12 + b13 + b17);
    fs[12] = f[12] + 0.25f * (b8 - b12 - b13 + b17);
    fs[13] = f[13] + 0.25f * (-b8 - b12 + b13 + b17);
    fs[14] = f[14] + 0.25f * (-b8 + b12 - b13 + b17);
    fs[15] = f[15] + 0.25f * (b9 + b14 + b15 + b18);
    fs[16] = f[16] + 0.25f * (b9 - b14 - b15 + b18);
    fs[17] = f[17] + 0.25f * (-b9 - b14 + b15 + b18);
    fs[18] = f[18] + 0.25f * (-b9 + b14 - b15 + b18);

    // recoloring (Eq. 10-11): F0_i = sum_k rho_k phi_i^k is rho_R alpha_R +
    // rho_B alpha_B at rest, p/6 on the axes and p/12 on the diagonals.
    // Stored red deviation: rho_R/rho f*_i + seg_i - R_R phi_i^R
    //   = (rho_R/rho) t_i + seg_i + cr_i,
    // cr_i = [R_R R_B (phi_i^B - phi_i^R) + eta_R R_B phi_i^B - eta_B R_R phi_i^R]/rho;
    // blue: t_i - (red deviation).  rho_R/rho is a correctly rounded
    // quotient (exactly 1 in a pure red node, so pure phases stay pure).
    const float ir = M.inv_rho;
    const float RR = s.R[0], RB = s.R[1];
    const float ar = RR / rho;
    const float bseg = C.beta * RR * RB * ir * ir;
    const float sa = bseg * p * (1.0f / 6.0f);
    const float rr = RR * RB;
    using P = typename S::P;
    const size_t N = (size_t)C.N, NS = (size_t)C.NS;
    if constexpr (OUT == LV_COMPACT) {
        // direction 0 as a pair, directions 1-18 as totals, the writer's data
        const float cr0 = (rr * (C.phi[1][0] - C.phi[0][0]) + s.eta[0] * RB * C.phi[1][0] -
                           s.eta[1] * RR * C.phi[0][0]) * ir;
        const float cr1 = (rr * (C.phi[1][1] - C.phi[0][1]) + s.eta[0] * RB * C.phi[1][1] -
                           s.eta[1] * RR * C.phi[0][1]) * ir;
        const uint32_t off = (uint32_t)node * (uint32_t)sizeof(T);
        T *tb = reinterpret_cast<T *>(a.fout) + C.pop_off;
        const float dr0 = ar * fs[0] + cr0;
        buf_st<P, CPS>(rsrc(tb, NS * sizeof(P)), (uint32_t)node * (uint32_t)sizeof(P),
                       P{S::enc(dr0, a.scale), S::enc(fs[0] - dr0, a.scale)});
        #pragma unroll
        for (int i = 1; i < Q; ++i)
            buf_st<T, CPS>(rsrc(tb + (size_t)(i + 1) * NS, NS * sizeof(T)), off, S::enc(fs[i], a.scale));
        buf_st<float2, CPS>(rsrc(a.rho_cur + C.node_off, N * sizeof(float2)), (uint32_t)node * 8u,
                            make_float2(RR, RB));
        buf_st<float4, CPS>(rsrc(a.dsc_cur + C.node_off, N * sizeof(float4)), (uint32_t)node * 16u,
                            make_float4(ar, sa * nx, sa * ny, sa * nz));
        buf_st<float, CPS>(rsrc(a.crs_cur + C.node_off, N * sizeof(float)), (uint32_t)node * 4u, cr1);
        return;
    }
    const float sd = bseg * p * (1.0f / 12.0f) * 0.70710678118654752f;
    float cr[3];
    #pragma unroll
    for (int k = 0; k < 3; ++k)
        cr[k] = (rr * (C.phi[1][k] - C.phi[0][k]) + s.eta[0] * RB * C.phi[1][k] - s.eta[1] * RR * C.phi[0][k]) * ir;
    float seg[Q];
    seg[0] = 0.f;
    seg[1] = sa * nx; seg[2] = -sa * nx; seg[3] = sa * ny; seg[4] = -sa * ny;
    seg[5] = sa * nz; seg[6] = -sa * nz;
    seg[7] = sd * (nx + ny); seg[8] = -seg[7]; seg[9] = sd * (nx - ny); seg[10] = -seg[9];
    seg[11] = sd * (nx + nz); seg[12] = -seg[11]; seg[13] = sd * (nx - nz); seg[14] = -seg[13];
    seg[15] = sd * (ny + nz); seg[16] = -seg[15]; seg[17] = sd * (ny - nz); seg[18] = -seg[17];

    P *outb = reinterpret_cast<P *>(a.fout) + C.pop_off / 2;
    #pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float dr = ar * fs[i] + seg[i] + cr[ecls(i)];
        const float db = fs[i] - dr;
        const uint32_t off = (uint32_t)node * (uint32_t)sizeof(P);
        buf_st<P, CPS>(rsrc(outb + (size_t)i * NS, NS * sizeof(P)), off, P{S::enc(dr, a.scale), S::enc(db, a.scale)});
    }
    buf_st<float2, CPS>(rsrc(a.rho_cur + C.node_off, N * sizeof(float2)), (uint32_t)node * 8u, make_float2(RR, RB));
}

// ------------------------------------------------------------- k_collide
template <int ST, bool MV, int WL>
__global__ __launch_bounds__(256) void k_collide(StepArgs a)
{
    const TileRange tr = tile_range(a.ntiles);
    for (int t = tr.first; t < tr.end; t += tr.stride) {
        const int2 tl = uniform_tile(a.tiles, t);
        DC &C = case_at(a.cases, tl.x);
        const int node = tl.y + (int)threadIdx.x;
        if (node >= C.N) continue;
        const Coord c = make_coord<WL>(C, node);
        NodeState s;
        pull_node<ST, MV>(a, C, c, s);
        Stencil st = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        stencil_acc(a, C, c, st);
        collide_node<ST>(a, C, node, s, st, a.aux[C.node_off + node].x);
    }
}

// ---------------------------------------------------------------- k_fused
// Single-pass step.  A workgroup owns an FTX x FTY tile of columns over a
// chunk of z-planes and marches up the chunk; each lane owns one column.  For
// plane z + 1 it pulls its own node, keeps the pulled state in registers and
// writes the node's aux value (rho^N, Qbar) into a four-plane LDS ring; a
// second round pulls the tile's one-node x-y halo for its aux values only.
// After one barrier the lanes collide plane z with the colour-gradient and
// correction stencils read from the ring, and the state of plane z + 1
// becomes the next plane's.  Populations are read once per node (the halo
// pulls of a tile's edge are the interior pulls of its neighbour, mostly
// served by the caches) and aux values never go to memory.  Walls, if any,
// lie on z: the ghost layer beyond a wall is computed in LDS from the first
// layer (wetting rule, Qbar reflected about its wall value), which needs that
// layer's phase field two nodes around the tile, so the wall layers are
// pulled with a two-node halo.  The four ring slots let one barrier per plane
// suffice: the slot written for plane z + 2 was last read by the collision of
// plane z - 2, which every lane finished before the previous barrier.
constexpr int FH = 2;                                  // halo width the ring can hold
constexpr int FRX = FTX + 2 * FH, FRY = FTY + 2 * FH, FREG = FRX * FRY;
constexpr int FSLOTS = 4;

struct FusedArgs {
    StepArgs a;
    const int4 *ftiles;          // (case, x0, y0, z0)
    int nftiles;
    int zc;                      // planes per chunk
};

__device__ inline int fslot(int z) { return (z + FSLOTS) & (FSLOTS - 1); }   // z >= -1
__device__ inline int fidx(int rx, int ry) { return (rx + FH) + FRX * (ry + FH); }

// aux value of a node from its pulled state; qs = sum_k rho_k (1 - 3 c_s^k^2)
__device__ inline float4 aux_value(DC &C, const NodeState &s, float &qs)
{
    const Macro m = macro(C, s);
    qs = s.R[0] * C.qc[0] + s.R[1] * C.qc[1];
    return make_float4(phase_field(C, s.R[0], s.R[1]), m.ux * qs, m.uy * qs, m.uz * qs);
}

__device__ inline int rslot(int z) { return (z + 4) & 3; }                 // z >= -4
__device__ inline int ridx(int rx, int ry) { return (rx + RH) + RW * (ry + RH); }

// Copy the stored densities of plane zl (the writers' densities of the level
// being pulled) around the tile into the LDS plane ring: the tile plus RH
// nodes on each side, which covers every pull source of the tile's nodes and
// of its halo.  Planes beyond a wall are not copied (their pulls bounce back).
// Split into the loads (RREG entries in two rounds over the workgroup's
// lanes, issued together and early) and the LDS stores, so that their
// latency hides behind the pulls issued in between.
// IN = LV_COMPACT: the writers' recoloring data are staged the same way into
// rings of their own.
template <int IN> struct RhoStage {
    float2 v[2];
    int d[2];
    float4 dv[IN == LV_COMPACT ? 2 : 1];
    float cv[IN == LV_COMPACT ? 2 : 1];
};

template <int IN>
__device__ inline RhoStage<IN> fused_stage_load(const StepArgs &a, DC &C, int zl, int x0, int y0, int ax, int ay,
                                                bool walls)
{
    RhoStage<IN> r;
    r.d[0] = r.d[1] = -1;
    int zp = zl;
    if (walls) {
        if (zl < 0 || zl >= C.nz) return r;
    } else {
        zp = (zl + 4 * C.nz) % C.nz;
    }
    static_assert(RREG <= 2 * FNT, "the writers' region must fit two rounds of the workgroup's lanes");
    const size_t pofs = (size_t)C.node_off + (size_t)C.nx * C.ny * zp;
    const int w = ax + 2 * RH, n = w * (ay + 2 * RH);
    #pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e0 = (int)threadIdx.x + FNT * k;
        const int e = min(e0, n - 1);                   // lanes past the region reload its last entry
        const int ry = e / w, rx = e - ry * w;
        // periodic wrap without branches (the region reaches RH < 4 nodes beyond the box)
        const int gx = (x0 + rx - RH + 4 * C.nx) % C.nx, gy = (y0 + ry - RH + 4 * C.ny) % C.ny;
        const size_t g = pofs + gx + (size_t)C.nx * gy;
        r.v[k] = a.rho_prev[g];
        if constexpr (IN == LV_COMPACT) {
            r.dv[k] = a.dsc_prev[g];
            r.cv[k] = a.crs_prev[g];
        }
        r.d[k] = e0 < n ? rx + RW * ry : -1;
    }
    return r;
}

template <int IN>
__device__ inline void fused_stage_store(float2 (*rring)[RREG], float4 *dring, float *cring, int zl,
                                         const RhoStage<IN> &r)
{
    float2 *dst = rring[rslot(zl)];
    #pragma unroll
    for (int k = 0; k < 2; ++k)
        if (r.d[k] >= 0) {
            dst[r.d[k]] = r.v[k];
            if constexpr (IN == LV_COMPACT) {
                dring[rslot(zl) * RREG + r.d[k]] = r.dv[k];
                cring[rslot(zl) * RREG + r.d[k]] = r.cv[k];
            }
        }
}

// Loaded values of one pull in the level format IN.
template <int ST, int IN> struct FPull;
template <int ST> struct FPull<ST, LV_PAIR> { typename Storage<ST>::P v[Q]; };
template <int ST> struct FPull<ST, LV_COMPACT> : CompactPull<ST> {};

template <int ST, int IN, int CPP, bool SO = false>
__device__ inline void fpull_issue(const StepArgs &a, DC &C, const Coord &c, FPull<ST, IN> &p)
{
    if constexpr (IN == LV_COMPACT) pull_issue_c<ST, CPP, SO>(a, C, c, p);
    else pull_issue<ST, CPP, SO>(a, C, c, p.v);
}

template <int ST, int IN, bool MV>
__device__ inline void fpull_finish(const StepArgs &a, DC &C, const Coord &c, const WriterRing &wr, int ri,
                                    const FPull<ST, IN> &p, NodeState &s)
{
    if constexpr (IN == LV_COMPACT) pull_finish_c<ST, MV>(a, C, c, wr, ri, p, s);
    else pull_finish<ST, MV>(a, C, c, wr.r, ri, p.v, s);
}

// Position (relative to the tile origin) of entry e of the halo of width h
// around an ax x ay tile: the 2h rows below and above (w = ax + 2h wide,
// nrow entries), then the 2h columns beside the tile.
__device__ inline void halo_pos(int e, int w, int nrow, int h, int ax, int ay, int &rx, int &ry)
{
    if (e < nrow) {
        const int r = e / w;
        rx = e - r * w - h;
        ry = r < h ? r - h : ay + (r - h);
    } else {
        const int e1 = e - nrow, cc = e1 / ay;
        ry = e1 - cc * ay;
        rx = cc < h ? cc - h : ax + (cc - h);
    }
}

// Position (relative to the tile origin) of entry e of the ring at distance
// exactly 2 around an ax x ay tile: the rows y = -2 and y = ay + 1 (ax + 4
// wide), then the columns x = -2 and x = ax + 1 (y = -1 .. ay).
__device__ inline void ring2_pos(int e, int ax, int ay, int &rx, int &ry)
{
    const int w = ax + 4;
    if (e < 2 * w) {
        const int r = e >= w;
        rx = e - r * w - 2;
        ry = r ? ay + 1 : -2;
    } else {
        const int e1 = e - 2 * w, r = e1 >= ay + 2;
        ry = e1 - r * (ay + 2) - 1;
        rx = r ? ax + 1 : -2;
    }
}

// The second halo ring of a wall layer (needed by the ghost layer's in-plane
// gradient): its writers lie beyond the LDS rings (RH = 2 nodes around the
// tile), so these pulls read the writers' words from memory (two planes per
// column of tiles).
template <int ST, bool MV, int WL, int IN>
__device__ inline void fused_ring2(const StepArgs &a, DC &C, float4 *slot, float (*wq)[FREG], bool wlo, bool whi,
                                   int zp, int x0, int y0, int ax, int ay)
{
    const int n = 2 * (ax + 4) + 2 * (ay + 2);
    for (int e = (int)threadIdx.x; e < n; e += FNT) {
        int rx, ry;
        ring2_pos(e, ax, ay, rx, ry);
        const int gx = (x0 + rx + 4 * C.nx) % C.nx, gy = (y0 + ry + 4 * C.ny) % C.ny;
        const Coord ch = make_coord_xyz<WL>(C, gx, gy, zp);
        NodeState hs;
        if constexpr (IN == LV_COMPACT) pull_node_c<ST, MV>(a, C, ch, hs);
        else pull_node<ST, MV, CP_DEFAULT>(a, C, ch, hs);
        float qs;
        slot[fidx(rx, ry)] = aux_value(C, hs, qs);
        if (wlo) wq[0][fidx(rx, ry)] = qs;
        if (whi) wq[1][fidx(rx, ry)] = qs;
    }
}

// Aux values of plane zp (0 <= zp < nz) into the ring slot of plane zl (zl =
// zp, or zp -+ nz for the periodic neighbours of the chunk's end planes): the
// lane's own node (pulled state kept in s) and the halo of width h (1, or 2
// on a wall layer).  The one-node halo (84 nodes around a 32 x 8 tile) is
// smaller than the workgroup, so a lane pulls at most one halo node; the
// halo duty falls on consecutive waves, rotated by plane.  Lanes outside a
// ragged tile (and past the halo) pull a valid node and drop the result.  On
// a wall layer of a case with moving walls the density factor qs of Qbar goes
// to wq[side] for the ghost layer.
template <int ST, bool MV, int WL, int IN, bool SO = false>
__device__ inline void fused_plane(const StepArgs &a, DC &C, float4 (*ring)[FREG], float2 (*rring)[RREG],
                                   const float4 *dring, const float *cring, float (*wq)[FREG], int zl, int zp,
                                   int x0, int y0, int ax, int ay, int h, bool active, int tx, int ty,
                                   NodeState &s)
{
    using P = typename Storage<ST>::P;
    float4 *slot = ring[fslot(zl)];
    const bool wlo = MV && C.wall == 2 && zp == 0, whi = MV && C.wall == 2 && zp == C.nz - 1;
    WriterRing wr;
    #pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int sl = rslot(zl - 1 + k);
        wr.r[k] = rring[sl];
        wr.d[k] = dring + (IN == LV_COMPACT ? sl * RREG : 0);
        wr.c[k] = cring + (IN == LV_COMPACT ? sl * RREG : 0);
    }
    // the one-node ring here; a wall layer's second ring after it (fused_ring2)
    const int w = ax + 2, nrow = 2 * w, nh = nrow + 2 * ay;
    const int rot = zl & (FNW - 1);
    const int e = ((int)threadIdx.x - 64 * rot + FNT) & (FNT - 1);
    const int wave = (int)threadIdx.x >> 6;
    const bool wave_halo = __builtin_amdgcn_readfirstlane((((wave - rot) & (FNW - 1)) * 64 < nh) ? 1 : 0) != 0;
    if constexpr (sizeof(P) == 8 && IN == LV_PAIR) {
        // FP32 pairs: a wave with halo duty issues both nodes' loads before it
        // waits (one memory latency instead of two, at 2 waves per SIMD)
        const int ox = min(tx, ax - 1), oy = min(ty, ay - 1);
        const Coord co = make_coord_xyz<WL>(C, x0 + ox, y0 + oy, zp);
        FPull<ST, IN> vo;
        fpull_issue<ST, IN, CP_DEFAULT, SO>(a, C, co, vo);
        float qs;
        if (wave_halo) {
            const int eh = min(e, nh - 1);
            int rx, ry;
            halo_pos(eh, w, nrow, 1, ax, ay, rx, ry);
            const int gx = (x0 + rx + 4 * C.nx) % C.nx, gy = (y0 + ry + 4 * C.ny) % C.ny;
            const Coord ch = make_coord_xyz<WL>(C, gx, gy, zp);
            FPull<ST, IN> vh;
            fpull_issue<ST, IN, CP_DEFAULT, SO>(a, C, ch, vh);
            __builtin_amdgcn_sched_barrier(0);   // both nodes' loads issued before the first use
            fpull_finish<ST, IN, MV>(a, C, co, wr, ridx(ox, oy), vo, s);
            if (active) {
                slot[fidx(tx, ty)] = aux_value(C, s, qs);
                if (wlo) wq[0][fidx(tx, ty)] = qs;
                if (whi) wq[1][fidx(tx, ty)] = qs;
            }
            NodeState hs;
            fpull_finish<ST, IN, MV>(a, C, ch, wr, ridx(rx, ry), vh, hs);
            if (e < nh) {
                slot[fidx(rx, ry)] = aux_value(C, hs, qs);
                if (wlo) wq[0][fidx(rx, ry)] = qs;
                if (whi) wq[1][fidx(rx, ry)] = qs;
            }
        } else {
            __builtin_amdgcn_sched_barrier(0);
            fpull_finish<ST, IN, MV>(a, C, co, wr, ridx(ox, oy), vo, s);
            if (active) {
                slot[fidx(tx, ty)] = aux_value(C, s, qs);
                if (wlo) wq[0][fidx(tx, ty)] = qs;
                if (whi) wq[1][fidx(tx, ty)] = qs;
            }
        }
    } else {
        // 16-bit forms and compact levels: the own node, then the halo node;
        // fewer registers (3 waves per SIMD for the 16-bit pairs), measured
        // faster for these forms
        float qs;
        if (active) {
            const Coord co = make_coord_xyz<WL>(C, x0 + tx, y0 + ty, zp);
            FPull<ST, IN> vo;
            fpull_issue<ST, IN, CP_DEFAULT, SO>(a, C, co, vo);
            __builtin_amdgcn_sched_barrier(0);
            fpull_finish<ST, IN, MV>(a, C, co, wr, ridx(tx, ty), vo, s);
            slot[fidx(tx, ty)] = aux_value(C, s, qs);
            if (wlo) wq[0][fidx(tx, ty)] = qs;
            if (whi) wq[1][fidx(tx, ty)] = qs;
        }
        for (int eh = e; eh < nh; eh += FNT) {
            int rx, ry;
            halo_pos(eh, w, nrow, 1, ax, ay, rx, ry);
            const int gx = (x0 + rx + 4 * C.nx) % C.nx, gy = (y0 + ry + 4 * C.ny) % C.ny;
            const Coord ch = make_coord_xyz<WL>(C, gx, gy, zp);
            FPull<ST, IN> vh;
            fpull_issue<ST, IN, CP_DEFAULT, SO>(a, C, ch, vh);
            __builtin_amdgcn_sched_barrier(0);
            NodeState hs;
            fpull_finish<ST, IN, MV>(a, C, ch, wr, ridx(rx, ry), vh, hs);
            slot[fidx(rx, ry)] = aux_value(C, hs, qs);
            if (wlo) wq[0][fidx(rx, ry)] = qs;
            if (whi) wq[1][fidx(rx, ry)] = qs;
        }
    }
    if (h == 2) fused_ring2<ST, MV, WL, IN>(a, C, slot, wq, wlo, whi, zp, x0, y0, ax, ay);
}

// Ghost layer beyond the wall at side `side` (0: z = -1, 1: z = nz) over the
// tile and its one-node halo, from the first layer's slot (which holds a
// two-node halo): rho^N follows the wetting rule with the 2D isotropic
// stencil, Qbar is reflected about its wall value (as k_ghost does).
template <bool MV>
__device__ inline void fused_ghost(DC &C, float4 (*ring)[FREG], float (*wq)[FREG], int side, int ax, int ay)
{
    const float4 *src = ring[fslot(side ? C.nz - 1 : 0)];
    float4 *dst = ring[fslot(side ? C.nz : -1)];
    const int w = ax + 2, n = w * (ay + 2);
    for (int e = (int)threadIdx.x; e < n; e += FNT) {
        const int ry = e / w - 1, rx = e - (ry + 1) * w - 1;
        float gb = 0.f, gc = 0.f;
        #pragma unroll
        for (int db = -1; db <= 1; ++db) {
            #pragma unroll
            for (int dc = -1; dc <= 1; ++dc) {
                if (db == 0 && dc == 0) continue;
                const float wgt = (db != 0 && dc != 0) ? (1.0f / 12.0f) : (1.0f / 3.0f);
                const float v = src[fidx(rx + db, ry + dc)].x;
                gb += wgt * (float)db * v;
                gc += wgt * (float)dc * v;
            }
        }
        const float4 s = src[fidx(rx, ry)];
        const float gpar = sqrtf(gb * gb + gc * gc);
        const float qw = MV && C.moving ? 2.0f * wq[side][fidx(rx, ry)] : 0.f;
        dst[fidx(rx, ry)] = make_float4(s.x + C.cot[side] * gpar, qw * C.uw[side][0] - s.y, qw * C.uw[side][1] - s.z,
                                        qw * C.uw[side][2] - s.w);
    }
}

template <int I = 1>
__device__ inline void stencil_lds(float4 (*ring)[FREG], int z, int tx, int ty, Stencil &st)
{
    if constexpr (I < Q) {
        constexpr int X = ex(I), Y = ey(I), Z = ez(I);
        constexpr float w3 = ecls(I) == 1 ? (1.0f / 6.0f) : (1.0f / 12.0f);
        const float4 v = ring[fslot(z + Z)][fidx(tx + X, ty + Y)];
        if constexpr (X != 0) { st.gx += (X * w3) * v.x; st.Qx += (X * w3) * v.y; }
        if constexpr (Y != 0) { st.gy += (Y * w3) * v.x; st.Qy += (Y * w3) * v.z; }
        if constexpr (Z != 0) { st.gz += (Z * w3) * v.x; st.Qz += (Z * w3) * v.w; }
        stencil_lds<I + 1>(ring, z, tx, ty, st);
    }
}

// WL: WALLS_NONE or WALLS_Z (cases with walls on other axes take the two-pass step).
// IN, OUT: level format read and written (LV_PAIR -> LV_PAIR, or -> LV_COMPACT;
// LV_COMPACT -> LV_COMPACT).
// SO: levels read through one buffer resource per case (the host takes it
// where every case's level is below 2^31 bytes).
template <int ST, bool MV, int WL, int IN, int OUT, bool SO = false>
__global__ __launch_bounds__(FNT) void k_fused(FusedArgs fa)
{
    __shared__ float4 ring[FSLOTS][FREG];
    __shared__ float2 rring[4][RREG];
    __shared__ float4 dring[IN == LV_COMPACT ? 4 * RREG : 1];
    __shared__ float cring[IN == LV_COMPACT ? 4 * RREG : 1];
    __shared__ float wq[MV ? 2 : 1][FREG];
    const StepArgs &a = fa.a;
    const TileRange tr = tile_range(fa.nftiles);
    const int tx = (int)threadIdx.x % FTX, ty = (int)threadIdx.x / FTX;
    for (int t = tr.first; t < tr.end; t += tr.stride) {
        const int4 tl = fa.ftiles[t];
        DC &C = case_at(a.cases, tl.x);
        const int x0 = tl.y, y0 = tl.z, z0 = tl.w;
        const int z1 = min(z0 + fa.zc, C.nz);
        const int ax = min(FTX, C.nx - x0), ay = min(FTY, C.ny - y0);
        const bool active = tx < ax && ty < ay;
        const bool walls = WL == WALLS_Z && C.wall == 2;
        __syncthreads();                                   // both rings reused across tiles
        // stored densities of the planes the prologue pulls read
        for (int q = z0 - 2; q <= z0 + 1; ++q)
            fused_stage_store<IN>(rring, dring, cring, q, fused_stage_load<IN>(a, C, q, x0, y0, ax, ay, walls));
        __syncthreads();
        NodeState cur, nxt;
        // plane z0 (kept) and the plane below it (the top plane, for a
        // periodic z at z0 = 0); at a bottom wall the ghost layer instead
        fused_plane<ST, MV, WL, IN, SO>(a, C, ring, rring, dring, cring, wq, z0, z0, x0, y0, ax, ay,
                                        walls && (z0 == 0 || z0 == C.nz - 1) ? 2 : 1, active, tx, ty, cur);
        if (!(walls && z0 == 0))
            fused_plane<ST, MV, WL, IN, SO>(a, C, ring, rring, dring, cring, wq, z0 - 1,
                                            z0 == 0 ? C.nz - 1 : z0 - 1, x0, y0, ax, ay, 1, active, tx, ty, nxt);
        __syncthreads();
        fused_stage_store<IN>(rring, dring, cring, z0 + 2,
                              fused_stage_load<IN>(a, C, z0 + 2, x0, y0, ax, ay, walls));
        if (walls && z0 == 0) fused_ghost<MV>(C, ring, wq, 0, ax, ay);
        __syncthreads();
        // Each plane: the aux values of plane z + 1 (or the top ghost layer),
        // the stored densities of plane z + 3 for the next plane's pulls, one
        // barrier, the collision of plane z.  The density slot written here
        // was last read by the pulls of plane z, before the previous barrier.
        for (int z = z0; z < z1; ++z) {
            const int zn = z + 1;
            const RhoStage<IN> rs = fused_stage_load<IN>(a, C, z + 3, x0, y0, ax, ay, walls);
            if (walls && zn == C.nz) {
                fused_ghost<MV>(C, ring, wq, 1, ax, ay);
            } else {
                const int zp = zn == C.nz ? 0 : zn;        // periodic wrap
                fused_plane<ST, MV, WL, IN, SO>(a, C, ring, rring, dring, cring, wq, zn, zp, x0, y0, ax, ay,
                                                walls && zp == C.nz - 1 ? 2 : 1, active, tx, ty, nxt);
            }
            fused_stage_store<IN>(rring, dring, cring, z + 3, rs);
            __syncthreads();
            if (active) {
                const int node = (x0 + tx) + C.nx * ((y0 + ty) + C.ny * z);
                Stencil st = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                stencil_lds(ring, z, tx, ty, st);
                // FP32 levels are stored non-temporally: the level is read
                // back only by the next step, and the caches then keep the
                // halo pulls of neighbouring tiles (measured +10 %); the 16-bit
                // forms measured faster with ordinary stores
                collide_node<ST, ST == LBCG_FP32 ? CP_STREAM : CP_DEFAULT, OUT>(a, C, node, cur, st,
                                                                               ring[fslot(z)][fidx(tx, ty)].x);
            }
            cur = nxt;
        }
    }
}

// ---------------------------------------------------------- diagnostics
// Macroscopic fields of one case plus deterministic FP64 partial sums per
// workgroup: {rho_R, rho_B, rho u_x, rho u_y, rho u_z, unstable-node count}.
template <int ST, int FMT>
__global__ __launch_bounds__(256) void k_moments(StepArgs a, int tile0, float *rR, float *rB, float *rN,
                                                 float *ux, float *uy, float *uz, double *partial)
{
    __shared__ double red[6][4];
    const int2 tl = a.tiles[tile0 + blockIdx.x];
    DC &C = case_at(a.cases, tl.x);
    const int node = tl.y + (int)threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (node < C.N) {
        const Coord c = make_coord(C, node);
        NodeState s;
        if constexpr (FMT == LV_COMPACT) pull_node_c<ST, true>(a, C, c, s);
        else pull_node<ST, true>(a, C, c, s);
        const Macro m = macro(C, s);
        if (rR) rR[node] = s.R[0];
        if (rB) rB[node] = s.R[1];
        if (rN) rN[node] = phase_field(C, s.R[0], s.R[1]);
        if (ux) ux[node] = m.ux;
        if (uy) uy[node] = m.uy;
        if (uz) uz[node] = m.uz;
        v[0] = (double)s.R[0] + (double)s.eta[0];
        v[1] = (double)s.R[1] + (double)s.eta[1];
        v[2] = (double)m.rho * m.ux; v[3] = (double)m.rho * m.uy; v[4] = (double)m.rho * m.uz;
        const bool bad = !(isfinite(s.R[0]) && isfinite(s.R[1]) && isfinite(m.ux) && isfinite(m.uy) &&
                           isfinite(m.uz)) || s.R[0] < C.neg_tol[0] || s.R[1] < C.neg_tol[1];
        v[5] = bad ? 1.0 : 0.0;
    }
    // wavefront reduction (64 lanes), then across the 4 wavefronts
    #pragma unroll
    for (int k = 0; k < 6; ++k)
        #pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        #pragma unroll
        for (int k = 0; k < 6; ++k) red[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int nw = (blockDim.x + 63) / 64;
        double acc = 0.0;
        for (int w = 0; w < nw; ++w) acc += red[threadIdx.x][w];
        partial[(size_t)blockIdx.x * 6 + threadIdx.x] = acc;
    }
}

// Sum n partial 6-vectors in a fixed order (one workgroup of 256 lanes).
__global__ __launch_bounds__(256) void k_reduce(const double *partial, int n, double *out)
{
    __shared__ double sh[6][256];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < n; b += blockDim.x)
        #pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] += partial[(size_t)b * 6 + k];
    #pragma unroll
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            #pragma unroll
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = sh[threadIdx.x][0];
}

// ------------------------------------------------------------ utilities
template <int I = 0>
__device__ inline void map_all(DC &C, const Coord &c, int64_t *sn, int8_t *sd)
{
    if constexpr (I < Q) {
        int src, dir;
        pull_source<I>(C, c, src, dir);
        sn[(size_t)I * C.N + c.node] = src;
        sd[(size_t)I * C.N + c.node] = (int8_t)dir;
        map_all<I + 1>(C, c, sn, sd);
    }
}

__global__ __launch_bounds__(256) void k_index_map(const DevCase *cases, int cid, int64_t *sn, int8_t *sd)
{
    DC &C = case_at(cases, cid);
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= C.N) return;
    map_all(C, make_coord(C, node), sn, sd);
}

// Current-level populations f_i^k(x) (the values the next collision sees):
// the pull of every direction, decoded to FP32.
template <int ST, int I = 0>
__device__ inline void get_dirs(const StepArgs &a, DC &C, const Coord &c, float *out)
{
    if constexpr (I < Q) {
        using S = Storage<ST>;
        using T = typename S::T;
        int src, dir;
        pull_source<I>(C, c, src, dir);
        const typename S::P *base = reinterpret_cast<const typename S::P *>(a.fin) + C.pop_off / 2;
        const size_t N = (size_t)C.N, NS = (size_t)C.NS;
        const float2 rp = a.rho_prev[C.node_off + src];
        const typename S::P v = base[(size_t)dir * NS + src];
        float vR = __builtin_fmaf(rp.x, C.phi[0][ecls(I)], S::dec(v.r, a.inv_scale));
        float vB = __builtin_fmaf(rp.y, C.phi[1][ecls(I)], S::dec(v.b, a.inv_scale));
        if constexpr (I != 0) {
            if (C.moving && dir != I) {   // bounce-back at a moving wall (src is this node)
                const float eu = wall_eu<I>(C, bounce_side<I>(c));
                vR = __builtin_fmaf(eu * C.wg[0][ecls(I) - 1], rp.x, vR);
                vB = __builtin_fmaf(eu * C.wg[1][ecls(I) - 1], rp.y, vB);
            }
        }
        out[(size_t)I * N + c.node] = vR;
        out[(size_t)(Q + I) * N + c.node] = vB;
        get_dirs<ST, I + 1>(a, C, c, out);
    }
}

// The same from a compact level: the red share of each value rebuilt from its
// writer's data.
template <int ST, int I = 0>
__device__ inline void get_dirs_c(const StepArgs &a, DC &C, const Coord &c, float *out)
{
    if constexpr (I < Q) {
        using S = Storage<ST>;
        using T = typename S::T;
        constexpr int cl = ecls(I);
        int src, dir;
        pull_source<I>(C, c, src, dir);
        const T *base = reinterpret_cast<const T *>(a.fin) + C.pop_off;
        const size_t N = (size_t)C.N, NS = (size_t)C.NS;
        const float2 rp = a.rho_prev[C.node_off + src];
        float vR, vB;
        if constexpr (I == 0) {
            const typename S::P v = reinterpret_cast<const typename S::P *>(base)[src];
            vR = __builtin_fmaf(rp.x, C.phi[0][0], S::dec(v.r, a.inv_scale));
            vB = __builtin_fmaf(rp.y, C.phi[1][0], S::dec(v.b, a.inv_scale));
        } else {
            const bool bb = dir != I;
            const float4 dw = a.dsc_prev[C.node_off + src];
            const float cw = a.crs_prev[C.node_off + src];
            const float t = S::dec(base[(size_t)(dir + 1) * NS + src], a.inv_scale);
            const float eg = e_dot<I>(dw);
            float seg = cl == 1 ? eg : kDiagSeg * eg;
            if (bb) seg = -seg;
            const float dR = __builtin_fmaf(dw.x, t, seg + (cl == 1 ? cw : 0.5f * cw));
            vR = __builtin_fmaf(rp.x, C.phi[0][cl], dR);
            vB = __builtin_fmaf(rp.y, C.phi[1][cl], t - dR);
            if (C.moving && bb) {   // bounce-back at a moving wall (src is this node)
                const float eu = wall_eu<I>(C, bounce_side<I>(c));
                vR = __builtin_fmaf(eu * C.wg[0][cl - 1], rp.x, vR);
                vB = __builtin_fmaf(eu * C.wg[1][cl - 1], rp.y, vB);
            }
        }
        out[(size_t)I * N + c.node] = vR;
        out[(size_t)(Q + I) * N + c.node] = vB;
        get_dirs_c<ST, I + 1>(a, C, c, out);
    }
}

template <int ST, int FMT>
__global__ __launch_bounds__(256) void k_get_pop(StepArgs a, int cid, float *out)
{
    DC &C = case_at(a.cases, cid);
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= C.N) return;
    if constexpr (FMT == LV_COMPACT) get_dirs_c<ST>(a, C, make_coord(C, node), out);
    else get_dirs<ST>(a, C, make_coord(C, node), out);
}

// Equilibrium start, Eq. (18) (improved) or Eq. (6) (original), evaluated in
// FP64 and rounded once into the storage format.  The buffers hold values that
// the next pull reads, so f_i^{k,eq}(y) is stored in the slot the pull of
// (y, i) reads: (src, dir) of pull_source, which is a permutation of all
// slots.  The slot at src holds the deviation from rho_k(src) phi_i^k.
struct InitCase { double alpha[2]; int improved; };

template <int ST, int I = 0>
__device__ inline void init_dirs(const StepArgs &a, DC &C, const Coord &c, const InitCase &ic,
                                 const double (&r)[2], const double (&u)[3], double uu, const double *rR0,
                                 const double *rB0)
{
    if constexpr (I < Q) {
        using S = Storage<ST>;
        using T = typename S::T;
        constexpr int cl = ecls(I);
        int src, dir;
        pull_source<I>(C, c, src, dir);
        T *base = reinterpret_cast<T *>(a.fout) + C.pop_off;
        const size_t NS = (size_t)C.NS;
        const double eu = ex(I) * u[0] + ey(I) * u[1] + ez(I) * u[2];
        const double w = cl == 0 ? 1.0 / 3.0 : (cl == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        #pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double al = ic.alpha[k];
            const double cs2 = 0.5 * (1.0 - al);
            const double ph = cl == 0 ? al : (cl == 1 ? (1.0 - al) / 12.0 : (1.0 - al) / 24.0);
            double br = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
            if (ic.improved) br += 3.0 * eu * (3.0 * cs2 - 1.0) * (3.0 * cl - 5.0);
            const double fe = r[k] * (ph + w * br);
            const float rs = (float)(k == 0 ? rR0[src] : rB0[src]);
            double dev = fe - (double)rs * (double)C.phi[k][cl];
            if constexpr (I != 0) {
                // a slot the pull reads across a moving wall gets the wall's
                // momentum added on the way; store the start level without it
                if (C.moving && dir != I)
                    dev -= (double)(wall_eu<I>(C, bounce_side<I>(c)) * C.wg[k][ecls(I) - 1]) * (double)rs;
            }
            base[((size_t)dir * NS + src) * 2 + k] = (T)(float)(dev * (double)a.scale);
        }
        init_dirs<ST, I + 1>(a, C, c, ic, r, u, uu, rR0, rB0);
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_init(StepArgs a, int cid, InitCase ic, const double *rR0,
                                              const double *rB0, const double *ux0, const double *uy0,
                                              const double *uz0)
{
    DC &C = case_at(a.cases, cid);
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= C.N) return;
    const double r[2] = {rR0[node], rB0[node]};
    const double u[3] = {ux0[node], uy0[node], uz0[node]};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    init_dirs<ST>(a, C, make_coord(C, node), ic, r, u, uu, rR0, rB0);
    a.rho_cur[C.node_off + node] = make_float2((float)r[0], (float)r[1]);
}

}  // namespace lbcg
