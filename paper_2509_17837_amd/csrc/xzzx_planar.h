// Building blocks of the packed-row kernels specialised to the planar
// lattice at distance D (odd, 3..15): the lattice turned by 45 degrees (rows
// of 2D + 1 columns, see PlanarSchedule), every row in registers for the
// whole run, the generator schedule in the instruction stream.  One chain per
// lane; a task's 64 chains may span syndromes (the paper's N_SA = 10 gives 40
// chains per syndrome), so the syndrome word of the Philox counter varies
// across the wavefront (planar_head and planar_philox_block).  Used by
// the annealing and the replica-exchange kernels of this lattice.
#pragma once

#include "xzzx_device.h"

namespace xzzx {

template <int D>
struct PlanarRows {
    static constexpr int R = 2 * D - 1;                        // rows
    static constexpr int C = 2 * D + 1;                        // columns (the last two are padding)
    static constexpr int NW = 2 * C <= 32 ? 1 : 2;             // words per row
    static constexpr int N = R * NW;                           // registers per chain
};

template <int D, int K, int B, int W>
struct PlanarGen {
    static constexpr RotGen g = kPlanarSchedule<D>.g[K][4 * B + W];
    static constexpr bool real = g.shp != 5;
    static constexpr int Y = g.Y, BO = g.bo;
};

// The move's energy-table entry from its 8-bit block pattern (top row, then
// bottom row).
template <int D, int K, int B, int W>
__device__ __forceinline__ uint4 planar_lookup(const uint32_t (&r)[PlanarRows<D>::N], const uint16_t *lut_s,
                                               const uint4 *et_s)
{
    using G = PlanarGen<D, K, B, W>;
    constexpr int NW = PlanarRows<D>::NW;
    if constexpr (!G::real) {
        return make_uint4(0u, 0u, 0u, 0u);
    } else {
        const uint32_t pat2 = (row_bits<NW, G::BO, 1>(r + G::Y * NW) & 0x1Eu) |
                              (row_bits<NW, G::BO, 5>(r + (G::Y + 1) * NW) & 0x1E0u);
        const uint32_t off = *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(lut_s) +
                                                                 512u * G::g.shp + pat2);
        return *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint8_t *>(et_s) + off);
    }
}

template <int D, int K, int B, int W>
__device__ __forceinline__ void planar_apply(uint32_t (&r)[PlanarRows<D>::N], uint32_t u, const uint4 &e, int32_t &acc)
{
    using G = PlanarGen<D, K, B, W>;
    constexpr int NW = PlanarRows<D>::NW;
    if constexpr (G::real) {
        const uint32_t sel = accept_sel(u, e.y, e.z);
        row_flip_static<NW, G::BO, 6u>(r + G::Y * NW, sel);         // X top-left | Z top-right
        row_flip_static<NW, G::BO, 9u>(r + (G::Y + 1) * NW, sel);   // Z bottom-left | X bottom-right
        acc += (int32_t)(e.x & sel);
    }
}

// Philox4x32-10 of the counter (uid, cc, c2, b) with uid and cc the lane's
// syndrome and chain, c2 and the key uniform across the wavefront and b the
// block.  Which words a product depends on: round 0 multiplies uid (fixed for
// the chain's whole run: PlanarLaneKey) and c2 (uniform); round 1 multiplies
// the word carrying cc (per sweep and class) and the one carrying uid and b
// (per block); round 2 multiplies the two words that follow from those.  The
// two products that do not involve b are taken once per sweep and class
// (planar_head); each block takes the other two, then rounds 3-9.
struct PlanarLaneKey {
    uint32_t hk1, w1;   // high word of M0*uid xor k1; low word of M0*uid
};

struct PlanarHead {
    uint32_t y1k;       // uniform: low word of M1*c2, xor the round-1 key k0 + W0
    uint32_t w2;        // lane: round-1 output w (low word of M0*x1)
    uint32_t a3, y3;    // lane: high and low words of M1*z2 (round 2)
};

__device__ __forceinline__ PlanarLaneKey planar_lane_key(uint32_t uid, uint32_t k1)
{
    const uint64_t p = (uint64_t)uid * kPhM0;
    return PlanarLaneKey{(uint32_t)(p >> 32) ^ k1, (uint32_t)p};
}

__device__ __forceinline__ PlanarHead planar_head(const PlanarLaneKey &lk, uint32_t cc, uint32_t c2, uint32_t k0,
                                                  uint32_t k1)
{
    PlanarHead h;
    const uint64_t p1 = (uint64_t)c2 * kPhM1;                  // round 0, uniform
    h.y1k = (uint32_t)p1 ^ (k0 + kPhW0);
    const uint32_t x1 = ((uint32_t)(p1 >> 32) ^ k0) ^ cc;     // lane
    const uint64_t q = (uint64_t)x1 * kPhM0;                   // round 1, lane
    const uint32_t z2 = xor3_key((uint32_t)(q >> 32), lk.w1, k1 + kPhW1);
    h.w2 = (uint32_t)q;
    const uint64_t r = (uint64_t)z2 * kPhM1;                   // round 2, lane
    h.a3 = (uint32_t)(r >> 32);
    h.y3 = (uint32_t)r;
    return h;
}

template <int B>
__device__ __forceinline__ uint4 planar_philox_block(const PlanarLaneKey &lk, const PlanarHead &h, uint32_t k0,
                                                     uint32_t k1)
{
    const uint32_t z1 = B == 0 ? lk.hk1 : lk.hk1 ^ (uint32_t)B;   // round 0 output z
    const uint64_t p1 = (uint64_t)z1 * kPhM1;                      // round 1
    const uint32_t x2 = (uint32_t)(p1 >> 32) ^ h.y1k;
    const uint64_t p0 = (uint64_t)x2 * kPhM0;                      // round 2
    uint4 c = make_uint4(xor3_key(h.a3, (uint32_t)p1, k0 + 2u * kPhW0), h.y3,
                         xor3_key((uint32_t)(p0 >> 32), h.w2, k1 + 2u * kPhW1), (uint32_t)p0);
    k0 += 3u * kPhW0;
    k1 += 3u * kPhW1;
#pragma unroll
    for (int i = 3; i < 10; ++i) {
        const uint64_t q0 = (uint64_t)c.x * kPhM0;
        const uint64_t q1 = (uint64_t)c.z * kPhM1;
        c = make_uint4(xor3_key((uint32_t)(q1 >> 32), c.y, k0), (uint32_t)q1,
                       xor3_key((uint32_t)(q0 >> 32), c.w, k1), (uint32_t)q0);
        k0 += kPhW0;
        k1 += kPhW1;
    }
    return c;
}

// The four moves of block B: entries looked up, then acceptance and flips.
template <int D, int K, int B>
__device__ __forceinline__ void planar_lookups(const uint32_t (&r)[PlanarRows<D>::N], const uint16_t *lut_s,
                                               const uint4 *et_s, uint4 (&e)[4])
{
    e[0] = planar_lookup<D, K, B, 0>(r, lut_s, et_s);
    e[1] = planar_lookup<D, K, B, 1>(r, lut_s, et_s);
    e[2] = planar_lookup<D, K, B, 2>(r, lut_s, et_s);
    e[3] = planar_lookup<D, K, B, 3>(r, lut_s, et_s);
}

template <int D, int K, int B>
__device__ __forceinline__ void planar_applies(uint32_t (&r)[PlanarRows<D>::N], const uint4 &u, const uint4 (&e)[4],
                                               int32_t &acc)
{
    planar_apply<D, K, B, 0>(r, u.x, e[0], acc);
    planar_apply<D, K, B, 1>(r, u.y, e[1], acc);
    planar_apply<D, K, B, 2>(r, u.z, e[2], acc);
    planar_apply<D, K, B, 3>(r, u.w, e[3], acc);
    asm("" : "+v"(acc));   // sum block by block (see static_block)
}

// Blocks B..NB-1 of a class, software-pipelined: the generators of one
// colour class act on disjoint qubits, so block B + 1's slots read the same
// before and after block B's flips, and its entries are looked up before
// those flips.  Its LDS round trips then overlap block B's acceptance
// instead of waiting for it (the register dependence through the rows would
// otherwise serialise the blocks; d = 9: 3 % faster).  The look-ahead's
// entries take registers: where they would spill at the kernel's occupancy
// (annealing d = 5, 11, 15; ladders also d = 7) the blocks run one after
// another.
constexpr bool planar_pipelined(int d) { return d != 5 && d != 11 && d != 15; }
constexpr bool planar_ladder_pipelined(int d) { return planar_pipelined(d) && d != 7; }

template <int D, int K, int B, int NB, bool PIPE>
__device__ __forceinline__ void planar_pipe(uint32_t (&r)[PlanarRows<D>::N], const PlanarLaneKey &lk,
                                            const PlanarHead &h, uint32_t k0, uint32_t k1, const uint16_t *lut_s,
                                            const uint4 *et_s, int32_t &acc, const uint4 (&e)[4])
{
    const uint4 u = planar_philox_block<B>(lk, h, k0, k1);
    if constexpr (B + 1 < NB && !PIPE) {
        planar_applies<D, K, B>(r, u, e, acc);
        uint4 en[4];
        planar_lookups<D, K, B + 1>(r, lut_s, et_s, en);
        planar_pipe<D, K, B + 1, NB, PIPE>(r, lk, h, k0, k1, lut_s, et_s, acc, en);
    } else if constexpr (B + 1 < NB) {
        uint4 en[4];
        planar_lookups<D, K, B + 1>(r, lut_s, et_s, en);
        planar_applies<D, K, B>(r, u, e, acc);
        planar_pipe<D, K, B + 1, NB, PIPE>(r, lk, h, k0, k1, lut_s, et_s, acc, en);
    } else {
        planar_applies<D, K, B>(r, u, e, acc);
    }
}

// One colour class of a sweep: c2 = 4t + k names the sweep and class in the
// Philox counter; PIPE: blocks software-pipelined.
template <int D, int K, bool PIPE>
__device__ __forceinline__ void planar_class(uint32_t (&r)[PlanarRows<D>::N], const PlanarLaneKey &lk, uint32_t cc,
                                             uint32_t c2, uint32_t k0, uint32_t k1, const uint16_t *lut_s,
                                             const uint4 *et_s, int32_t &acc)
{
    constexpr int NB = PlanarSchedule<D>::MP / 4;
    const PlanarHead h = planar_head(lk, cc, c2, k0, k1);
    uint4 e[4];
    planar_lookups<D, K, 0>(r, lut_s, et_s, e);
    planar_pipe<D, K, 0, NB, PIPE>(r, lk, h, k0, k1, lut_s, et_s, acc, e);
}

// qubit at row Y, column C of the turned lattice, or -1
template <int D>
__device__ __forceinline__ int planar_qubit_at(int Y, int C)
{
    const int u = Y + 1, v = C - (D - 1);
    return PlanarSchedule<D>::qubit(u + v + 1, u - v);
}

// The chain's starting state packed into the turned rows (the logical
// operators of its coset applied as asked), and its energy.
template <int D>
__device__ __forceinline__ int32_t planar_load(const PlanDev *pl, const ChainJob &J, bool use_x, bool use_z,
                                               const int32_t (&W)[4], uint32_t (&r)[PlanarRows<D>::N])
{
    using PR = PlanarRows<D>;
    constexpr int NW = PR::NW;
    int32_t E = 0;
#pragma unroll
    for (int Y = 0; Y < PR::R; ++Y) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t word = 0;
            if (J.active) {
#pragma unroll 1
                for (int C = 16 * w; C < min(PR::C, 16 * w + 16); ++C) {
                    const int q = planar_qubit_at<D>(Y, C);
                    if (q < 0) continue;
                    uint32_t v = J.src[q] & 3u;
                    if (use_x) v ^= pl->lx[q];
                    if (use_z) v ^= pl->lz[q];
                    word |= v << (2 * (C - 16 * w));
                    E += weight_of(W, v);
                }
            }
            r[Y * NW + w] = word;
        }
    }
    return E;
}

// One byte per qubit (the lattice's qubit order) from the turned rows.
template <int D>
__device__ __forceinline__ void planar_unpack(const uint32_t (&r)[PlanarRows<D>::N], uint8_t *dst)
{
    using PR = PlanarRows<D>;
    constexpr int NW = PR::NW;
#pragma unroll
    for (int Y = 0; Y < PR::R; ++Y)
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll 1
            for (int C = 16 * w; C < min(PR::C, 16 * w + 16); ++C) {
                const int q = planar_qubit_at<D>(Y, C);
                if (q >= 0) dst[q] = (uint8_t)((r[Y * NW + w] >> (2 * (C - 16 * w))) & 3u);
            }
}

// The rows of a chain, stored with 16-byte stores from one base address
// (NP = the rows padded to a multiple of four words).
template <int N>
__device__ __forceinline__ void store_rows(uint4 *dst, const uint32_t (&r)[N])
{
    constexpr int NP = (N + 3) / 4 * 4;
#pragma unroll
    for (int i = 0; i < NP / 4; ++i)
        dst[i] = make_uint4(r[4 * i], 4 * i + 1 < N ? r[4 * i + 1] : 0u, 4 * i + 2 < N ? r[4 * i + 2] : 0u,
                            4 * i + 3 < N ? r[4 * i + 3] : 0u);
}

// wavefronts per SIMD (VGPR budget 512 / waves): the rows take 2D - 1
// registers (one word per row, d <= 7) or 2(2D - 1), beside the lane-varying
// Philox words and the look-ahead entries; the most waves that compile
// without spills (at d = 9 five waves spill a few registers and measured 3-6 %
// slower than four)
constexpr int planar_waves(int d) { return d <= 5 ? 8 : d == 7 ? 6 : d == 9 ? 4 : d == 11 ? 4 : 3; }

}  // namespace xzzx
