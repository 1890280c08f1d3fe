// gm_common.h -- constants and small device helpers for the gfx950 path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GM_HD __host__ __device__ __forceinline__
#define GM_D __device__ __forceinline__

namespace gm {

// CGS constants (CODATA 2018).
constexpr double kC = 2.99792458e10;       // cm/s
constexpr double kH = 6.62607015e-27;      // erg s
constexpr double kE = 4.80320471e-10;      // esu
constexpr double kMe = 9.1093837015e-28;   // g
constexpr double kSigT = 6.6524587321e-25; // cm^2
constexpr double kMeC2 = kMe * kC * kC;    // erg
constexpr double kPi = 3.14159265358979323846;

// Hot cross-section table: 64 nodes in ln Theta on [1e-2, 1e3], 256 in
// ln eps on [1e-12, 1e6].
constexpr int kShNT = 64;
constexpr int kShNE = 256;
constexpr double kShThMin = 1e-2, kShThMax = 1e3;
constexpr double kShEMin = 1e-12, kShEMax = 1e6;

// Holds a loaded value in a register at this point of the program.  Loads
// whose results are all settled together are issued as one batch and waited
// for once; otherwise the compiler may sink some of them past a branch or
// reuse their registers, paying the memory latency once per round.
GM_D void settle(double v) { asm volatile("" :: "v"(v)); }
GM_D void settle(float v) { asm volatile("" :: "v"(v)); }

// Rejection loops stop after this many trials.
constexpr int64_t kMaxTrials = 100000;
// Margin on the per-zone frequency rejection bound (curvature of ln J
// between weight nodes).
constexpr double kFmaxMargin = 1.02;

// Ledger and statistics slots (same numbering as the public header).
enum { L_W_EMIT = 0, L_E_EMIT, L_W_ESC, L_E_ESC, L_W_OOB, L_E_OOB, L_W_ABS, L_E_ABS,
       L_W_CAPT, L_E_CAPT, L_W_CAPLOSS, L_E_CAPLOSS, L_W_ROUL, L_E_ROUL, L_W_STUCK, L_E_STUCK,
       L_E_COMPTON, L_E_DRIFT, L_N };
enum { S_ROOTS = 0, S_CHILDREN, S_STEPS, S_VERLET_IT, S_SCATTER, S_ROUL_KILL, S_ROUL_SURVIVE,
       S_CAPTURED, S_ESCAPED, S_OOB, S_STUCK, S_OVERSHOOT, S_NU_TRIALS, S_DIR_TRIALS,
       S_E_TRIALS, S_ANG_TRIALS, S_GEN0, S_COEF = S_GEN0 + 16, S_N };
enum { END_ESCAPE = 1, END_OOB, END_CAPTURE, END_ROULETTE, END_STUCK, END_SPLIT };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Ten rounds of two
// 32x32->64 multiplies with the Weyl key schedule.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

GM_HD U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// A photon's random stream: counter (block, s0, s1, s2), key = seed.  Each
// block gives one uniform in [0,1) from the first two words (53 bits).
struct Rng {
    uint32_t s0, s1, s2, block;
};

GM_HD double rng_uniform(Rng &r, uint32_t k0, uint32_t k1)
{
    U4 o = philox10(U4{r.block, r.s0, r.s1, r.s2}, k0, k1);
    r.block += 1;
    uint64_t bits = ((uint64_t)o.x << 21) | (uint64_t)(o.y >> 11);
    return (double)bits * 0x1.0p-53;
}

// Child stream: Philox under key (seed_lo ^ 0x9E3779B9, seed_hi) on
// (parent block at the scattering, parent stream); top bit of the third
// word set (roots use instance<<8|1, zone draws instance<<8|2).
GM_HD Rng child_rng(const Rng &p, uint32_t block_at, uint32_t k0, uint32_t k1)
{
    U4 o = philox10(U4{block_at, p.s0, p.s1, p.s2}, k0 ^ 0x9E3779B9u, k1);
    return Rng{o.x, o.y, o.z | 0x80000000u, 0u};
}

// Value of a per-zone table at log variable v: n nodes per zone uniform in
// v over [lo, hi], linear between nodes, the end node's value outside.
GM_HD double zone_table(const double *tab, int n, double lo, double hi, int z, double v)
{
    const double *t = tab + (size_t)z * n;
    double pos = (v - lo) / (hi - lo) * (double)(n - 1);
    if (pos <= 0.0) return t[0];
    if (pos >= (double)(n - 1)) return t[n - 1];
    int i = (int)floor(pos);
    double f = pos - (double)i;
    return t[i] + f * (t[i + 1] - t[i]);
}

// No event record (event-log index of a photon without one).
constexpr uint32_t kNoEvent = 0xffffffffu;

// Keep a wave-uniform value in a vector register: the compiler otherwise
// re-reads kernel arguments from memory inside long loops when scalar
// registers run short, and waits for every re-read.
GM_D void keep_vgpr(double &x) { asm volatile("" : "+v"(x)); }
GM_D void keep_vgpr(int &x) { asm volatile("" : "+v"(x)); }
GM_D void keep_vgpr(uint32_t &x) { asm volatile("" : "+v"(x)); }

// ---------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------
GM_D int lane_id() { return (int)__lane_id(); }

GM_D uint32_t rank_in_mask(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

GM_D uint64_t bcast_u64(uint64_t v, int src)
{
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace gm
