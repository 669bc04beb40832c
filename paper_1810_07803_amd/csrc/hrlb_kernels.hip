// hrlb_kernels.hip -- gfx950 kernels of the half-range lattice Boltzmann Couette solver.
//
// Per Runge-Kutta stage two launches cover every instance of a batch:
//   stage_kernel  one pass over (cell, velocity) units: WENO-5 face values of the stage input
//                 (diffuse-wall ghosts at the channel ends), reduced Shakhov collision, the SSP-RK3
//                 stage combine, the store of the stage output, and FP64 partial sums of that
//                 output's moments (and optionally residual), reduced per tile in LDS in a fixed
//                 order.
//   cell_kernel   per cell: sums the partials over velocity groups, forms the moments of Sec. II,
//                 the relaxation time of eq. (tau), the Shakhov prefactor and the truncated
//                 equilibria of eqs. (gx), (gy) that the next stage's collision uses; per instance:
//                 the leaving wall fluxes and the wall densities of eq. (diffuse_nw).
// The half channel (point symmetry of Sec. II) replaces the left wall by ghosts read from the
// mirrored velocities of the first cells.  Around the step: finalize_kernel (residual, channel mean
// of P_xy, mass at a checked step), renorm_kernel (local time steps: back to the rest-state mass
// after a check), average_kernel (time averages), init_kernel (rest equilibrium).
// Layout: populations [dist][v][cell] with cells contiguous.  A thread owns 4 consecutive cells of
// one velocity and reconstructs their 5 faces from a 12-cell window (the right face is also the
// next thread's left face; recomputing it costs less than fetching it: a per-tile pre-pass that
// read the tile-edge cells once more cost 20% extra HBM reads).  A block covers 64 cells x 16
// velocity rows; the tile's cell tables (moments, equilibria) are staged in LDS.  With FP32 storage
// each wave's loads for its next velocity go straight from the buffer unit into LDS while it
// computes the current one.
#include "hrlb_internal.h"
#include "hrlb_math.h"

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>


namespace hrlb {

// FLAG_FIELDS: the per-cell kernel also stores the FP64 fields (always at the end of a step, with
// FLAG_STEP_DONE; analysis passes ask for them; the stages inside a step do not need them)
enum : int { FLAG_RESID = 1, FLAG_STEP_DONE = 2, FLAG_FIELDS = 4 };

// Loads and stores through the global address space (the pointers live in descriptors, so the
// compiler would otherwise emit flat instructions).
#if defined(__HIP_DEVICE_COMPILE__)
#define HRLB_GLOBAL __attribute__((address_space(1)))
#else
#define HRLB_GLOBAL
#endif
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));

// ---- loads / stores of 2 consecutive cells -----------------------------------------------------
__device__ __forceinline__ void ld2(const float* p, float& a, float& b)
{
    const f2v v = *(const HRLB_GLOBAL f2v*)p;
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void ld2(const double* p, double& a, double& b)
{
    const d2v v = *(const HRLB_GLOBAL d2v*)p;
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void st2(float* p, float a, float b)
{
    f2v v;
    v.x = a;
    v.y = b;
    *(HRLB_GLOBAL f2v*)p = v;
}
__device__ __forceinline__ void st2(double* p, double a, double b)
{
    d2v v;
    v.x = a;
    v.y = b;
    *(HRLB_GLOBAL d2v*)p = v;
}
template <typename T>
__device__ __forceinline__ T gld(const T* p) { return *(const HRLB_GLOBAL T*)p; }
// the same pointer in the global address space: its accesses count on the vector memory counter
// alone, so that waits for LDS reads do not also wait for them (flat accesses count on both)
template <typename T>
using gptr = HRLB_GLOBAL T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) { return (gptr<T>)p; }

__device__ __forceinline__ float rcp6(float den) { return __builtin_amdgcn_rcpf(6.0f * den); }
// FP64: the hardware reciprocal refined by two Newton-Raphson steps (r <- r + r (1 - x r)), which
// square its relative error each; within an ulp or so of the quotient, for the positive normal
// denominators of the WENO weights (at least about 1e-21 from the smoothness floor), at about half
// the instructions of the IEEE division sequence
__device__ __forceinline__ double rcp6(double den)
{
    const double x = 6.0 * den;
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// ---- WENO-5 (Jiang & Shu) in difference form ----------------------------------------------------
// With the cells ordered along the upwind direction (a, b, c, d, e; c the upwind cell):
//   dm = c - b, dp = d - c, d2m = a - 2b + c, d2c = b - 2c + d, d2p = c - 2d + e,
//   E_x = 13/12 d2x^2 + eps,
//   beta0 = E_m + (d2m + 2 dm)^2/4, beta1 = E_c + (dm + dp)^2/4, beta2 = E_p + (d2p - 2 dp)^2/4,
//   candidate values q_k = c + y_k/6 with y0 = 2 d2m + 3 dm, y1 = dm + 2 dp, y2 = 3 dp - d2p,
//   weights 0.1, 0.6, 0.3 over (eps + beta_k)^2, normalised.
// The code carries t_k = 4 (eps + beta_k) (em, ec, ep hold 4 E_x): the common factor cancels in
// the normalised weights and saves a multiplication per indicator.
// Contraction is off so that every call site produces the same bits from the same inputs.
#pragma clang fp contract(off)
template <typename T>
__device__ __forceinline__ T weno_d(T c, T dm, T dp, T d2m, T d2p, T em, T ec, T ep)
{
    const T x0 = fma(T(2), dm, d2m);
    const T x1 = dm + dp;
    const T x2 = fma(T(-2), dp, d2p);
    const T t0 = fma(x0, x0, em);
    const T t1 = fma(x1, x1, ec);
    const T t2 = fma(x2, x2, ep);
    const T u0 = t0 * t0, u1 = t1 * t1, u2 = t2 * t2;
    const T a0 = u1 * u2, a1 = T(6) * (u0 * u2), a2 = T(3) * (u0 * u1);
    const T y0 = fma(T(2), d2m, T(3) * dm);
    const T y1 = fma(T(2), dp, dm);
    const T y2 = fma(T(3), dp, -d2p);
    const T num = fma(a2, y2, fma(a1, y1, a0 * y0));
    const T den = (a0 + a1) + a2;
    return fma(num, rcp6(den), c);
}

// 4 (13/12 d2^2 + eps), the scaled smoothness term of weno_d
template <typename T>
__device__ __forceinline__ T e_of(T d2) { return fma(T(13.0 / 3.0) * d2, d2, T(4e-6)); }

// face value from five cells in upwind order (used where no shared differences are at hand)
template <typename T>
__device__ __forceinline__ T weno5_cells(T a, T b, T c, T d, T e)
{
    const T dma = b - a, dm = c - b, dp = d - c, dpp = e - d;
    const T d2m = dm - dma, d2c = dp - dm, d2p = dpp - dp;
    return weno_d(c, dm, dp, d2m, d2p, e_of(d2m), e_of(d2c), e_of(d2p));
}

// Quadratic extrapolation (in cell index) through the three cells next to a wall (nodes at 0, 1, 2),
// used for ghosts of directions leaving the domain.
template <typename T>
__device__ __forceinline__ T ext_p3(T y0, T y1, T y2) { return (y0 - T(3) * y1) + T(3) * y2; }         // t = 3
template <typename T>
__device__ __forceinline__ T ext_p4(T y0, T y1, T y2) { return (T(3) * y0 - T(8) * y1) + T(6) * y2; }  // t = 4
template <typename T>
__device__ __forceinline__ T ext_m1(T y0, T y1, T y2) { return (T(3) * y0 - T(3) * y1) + y2; }         // t = -1
template <typename T>
__device__ __forceinline__ T ext_m2(T y0, T y1, T y2) { return (T(6) * y0 - T(8) * y1) + T(3) * y2; }  // t = -2

// leaving face value at the left wall (p_x < 0) from cells 0, 1, 2 with extrapolated ghosts -1, -2
template <typename T>
__device__ __forceinline__ T wall_face_left(T f0, T f1, T f2)
{
    return weno5_cells(f2, f1, f0, ext_m1(f0, f1, f2), ext_m2(f0, f1, f2));
}
// leaving face value at the right wall (p_x > 0) from cells nx-3, nx-2, nx-1 with ghosts nx, nx+1
template <typename T>
__device__ __forceinline__ T wall_face_right(T fa, T fb, T fc)
{
    return weno5_cells(fa, fb, fc, ext_p3(fa, fb, fc), ext_p4(fa, fb, fc));
}
#pragma clang fp contract(on)

// counter-based 32-bit hash (integer avalanche "lowbias32", C. Wellons, 2018)
__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// successor of a hashed word for the neighbouring cell of a strip: a Weyl step by the 32-bit golden
// ratio constant (one addition).  Each word stays uniform, so each rounding stays unbiased; the words
// of the 4 cells of a strip are evenly spread rather than independent.
__device__ __forceinline__ uint32_t weyl32(uint32_t x) { return x + 0x9e3779b9u; }

// Stochastic rounding of an FP64 value to FP32 with 16 random bits: the 29 bits a conversion
// drops are incremented by r << 13 before truncation, so the value rounds away from zero with
// probability equal to its dropped fraction (resolution 2^-16 ulp).
__device__ __forceinline__ float round_stochastic(double x, uint32_t r16)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    b += (unsigned long long)(r16 & 0xffffu) << 13;
    b &= ~0x1fffffffull;
    return (float)__longlong_as_double((long long)b);
}

template <typename T>
__device__ __forceinline__ T store_round(double x, int stochastic, uint32_t r16);
template <>
__device__ __forceinline__ double store_round<double>(double x, int, uint32_t) { return x; }
template <>
__device__ __forceinline__ float store_round<float>(double x, int stochastic, uint32_t r16)
{
    return stochastic ? round_stochastic(x, r16) : (float)x;
}

// the value of x in the partner lane of a DPP pattern within a 16-lane row (both 32-bit halves).  Every
// pattern used here reads a valid lane of the same row for every lane, so no lane keeps its old value
// and the moves need none (no register to initialise first).
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// sum over the 64 lanes of a wave, the same bits in every lane: a butterfly whose in-row steps take
// their partners from DPP patterns (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror; every lane of a group holds the same value after the steps before it), then the two
// steps across 16-lane rows through LDS permutes
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_partner<0xB1>(x);
    x += dpp_partner<0x4E>(x);
    x += dpp_partner<0x141>(x);
    x += dpp_partner<0x140>(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// ---- buffer resources: 32-bit byte offsets from a base held in scalar registers ---------------
typedef float f4v __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));
constexpr int kBufDword3 = 0x00020000;  // raw (untyped) buffer access on gfx9-family targets

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kBufDword3);
}
// four consecutive values at byte offset off + soff (16-byte aligned for float, two 16-byte loads for
// double); soff is the wave-uniform part of the offset, which the instruction adds from a scalar register
__device__ __forceinline__ void bld4(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[4], uint32_t soff = 0)
{
    const f4v v = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)soff, 0));
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
}
__device__ __forceinline__ void bld4(__amdgpu_buffer_rsrc_t r, uint32_t off, double (&o)[4], uint32_t soff = 0)
{
    const d2v a = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)soff, 0));
    const d2v b = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off + 16, (int)soff, 0));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
__device__ __forceinline__ void bst4(__amdgpu_buffer_rsrc_t r, uint32_t off, const float (&o)[4], uint32_t soff = 0)
{
    f4v v;
    v.x = o[0];
    v.y = o[1];
    v.z = o[2];
    v.w = o[3];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i4v, v), r, (int)off, (int)soff, 0);
}
__device__ __forceinline__ void bst4(__amdgpu_buffer_rsrc_t r, uint32_t off, const double (&o)[4], uint32_t soff = 0)
{
    d2v a, b;
    a.x = o[0];
    a.y = o[1];
    b.x = o[2];
    b.y = o[3];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i4v, a), r, (int)off, (int)soff, 0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i4v, b), r, (int)off + 16, (int)soff, 0);
}
template <typename T>
__device__ __forceinline__ T bld1(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bld1<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double bld1<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// ---- prefetch through LDS (FP32 stage kernel) ----------------------------------------------------
// The buffer unit writes a velocity's 16-byte loads of a wave straight into that wave's LDS buffer:
// slot i of lane l lands at buf + i kPfLoad + 16 l.  Slots: the windows of phi (cells s0-4.., s0..,
// s0+4..) and of chi, then the previous stage's values f^n of phi and chi at cells s0...  The loads
// of the next velocity are in flight while the wave computes the current one, and they hold no
// registers meanwhile.  The velocity loop issues no other vector-memory load, so the only waits on
// the memory counter are the ones below.
constexpr int kPfSlots = 8;
constexpr int kPfLoad = 64 * 16;                   // bytes of one slot of a wave
constexpr int kPfWave = kPfSlots * kPfLoad;        // bytes of a wave's buffer
typedef __attribute__((address_space(3))) void* lds_ptr;

__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t r, unsigned char* slot, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)slot, 16, voff, soff, 0, 0);
}

// Reads slots 0..N-1 of the lane (LDS byte address la) once at most W vector-memory operations of
// the wave are outstanding; the memory counter retires in issue order.  The reads are complete when
// the statement ends (their results are not used before).
template <int W, int N>
__device__ __forceinline__ void read_slots(uint32_t la, f4v (&t)[kPfSlots])
{
    static_assert((W == 0 || W == 2) && (N == 6 || N == 8), "read_slots: W in {0, 2}, N in {6, 8}");
#define HRLB_RD6                                                                                      \
    "ds_read_b128 %0, %8\n\tds_read_b128 %1, %8 offset:1024\n\tds_read_b128 %2, %8 offset:2048\n\t"      \
    "ds_read_b128 %3, %8 offset:3072\n\tds_read_b128 %4, %8 offset:4096\n\tds_read_b128 %5, %8 offset:5120\n\t"
#define HRLB_RD8 HRLB_RD6 "ds_read_b128 %6, %8 offset:6144\n\tds_read_b128 %7, %8 offset:7168\n\t"
#define HRLB_OUTS                                                                                     \
    "=&v"(t[0]), "=&v"(t[1]), "=&v"(t[2]), "=&v"(t[3]), "=&v"(t[4]), "=&v"(t[5]), "=&v"(t[6]), "=&v"(t[7])
    if constexpr (W == 0 && N == 6)
        __asm__ volatile("s_waitcnt vmcnt(0)\n\t" HRLB_RD6 "s_waitcnt lgkmcnt(0)" : HRLB_OUTS : "v"(la));
    else if constexpr (W == 2 && N == 6)
        __asm__ volatile("s_waitcnt vmcnt(2)\n\t" HRLB_RD6 "s_waitcnt lgkmcnt(0)" : HRLB_OUTS : "v"(la));
    else if constexpr (W == 0 && N == 8)
        __asm__ volatile("s_waitcnt vmcnt(0)\n\t" HRLB_RD8 "s_waitcnt lgkmcnt(0)" : HRLB_OUTS : "v"(la));
    else
        __asm__ volatile("s_waitcnt vmcnt(2)\n\t" HRLB_RD8 "s_waitcnt lgkmcnt(0)" : HRLB_OUTS : "v"(la));
#undef HRLB_RD6
#undef HRLB_RD8
#undef HRLB_OUTS
}
// Wait until no vector-memory operation of the wave is outstanding.
__device__ __forceinline__ void vm_drain() { __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// moments reduced per pass of the stage kernel's epilogue in the dynamic LDS: 2 for FP32 storage
// (the block's LDS share also holds the prefetch buffers; only the analysis kernel reduces there,
// the step kernels reduce 4 per pass in their drained prefetch buffers), 4 for FP64
__host__ __device__ constexpr int moments_per_pass(size_t elem) { return elem == 4 ? 2 : kMomPerPass; }

// The window of a thread owning cells s0..s0+3 is w[m] = cell s0 - 4 + m, m = 0..11; its faces
// f = 0..4 lie between cells s0+f-1 and s0+f (face 4 is also the next thread's face 0: both are
// formed from the same five cells in the same order, so they agree bit for bit).
// Differences: dl[m] = w[m+1] - w[m], d2[m] = dl[m] - dl[m-1].
template <typename T>
struct Win {
    T w[12];
    T dl[10], d2[10], e[10];
    // p_x > 0: face f has upwind cell C = f + 3 and needs dl[1..8], d2[2..8]
    __device__ __forceinline__ void faces_pos(T (&F)[5])
    {
#pragma unroll
        for (int m = 1; m <= 8; ++m) dl[m] = w[m + 1] - w[m];
#pragma unroll
        for (int m = 2; m <= 8; ++m) {
            d2[m] = dl[m] - dl[m - 1];
            e[m] = e_of(d2[m]);
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const int C = f + 3;
            F[f] = weno_d(w[C], dl[C - 1], dl[C], d2[C - 1], d2[C + 1], e[C - 1], e[C], e[C + 1]);
        }
    }
    // p_x < 0: face f has upwind cell C = f + 4 (cells mirrored) and needs dl[2..9], d2[3..9]
    __device__ __forceinline__ void faces_neg(T (&F)[5])
    {
#pragma unroll
        for (int m = 2; m <= 9; ++m) dl[m] = w[m + 1] - w[m];
#pragma unroll
        for (int m = 3; m <= 9; ++m) {
            d2[m] = dl[m] - dl[m - 1];
            e[m] = e_of(d2[m]);
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const int C = f + 4;
            F[f] = weno_d(w[C], -dl[C], -dl[C - 1], d2[C + 1], d2[C - 1], e[C + 1], e[C], e[C - 1]);
        }
    }
};

// Per-tile staging of the cell tables in LDS: the FP64 per-cell scalars, then (storage precision)
// 1/(J deta), g_y for every j of the instance, and g_x of the block's 16 rows.  Inside a slot the 64
// cells are stored as [4 cells of a thread][16 threads of a row], so that the 16 lanes of a row read
// 16 consecutive words; slots are kLdsSlot elements apart, which puts the 4 rows of a wave (reading
// slots one apart for g_x) on disjoint bank ranges.
// The FP64 scalar slots are read at the same slot by every row (broadcast), so they are packed
// kTileCells apart.
__host__ __device__ constexpr int g_lds_slots(int qy) { return 1 + qy + kRows; }
constexpr int kLdsSlot = kTileCells + kTPR;
constexpr int kScSlot = kTileCells;
__host__ __device__ constexpr size_t cell_lds_bytes(int qy, size_t es)
{
    return sizeof(double) * kNSc * kScSlot + es * (size_t)g_lds_slots(qy) * kLdsSlot;
}

// MODE: kModeAnalyze (no update; partials of the current state f[0], used after set-up or a state
// upload), kModeStep0 (the first stage of a step, which reads no f^n), kModeStep (stage 2 or 3),
// kModeResid (a stage 3 that also forms the residual partials)
enum : int { kModeAnalyze = 0, kModeStep0 = 1, kModeStep = 2, kModeResid = 3 };
// Work distribution: one queue per XCD.  Block b runs on XCD b % 8 (blocks are dispatched round
// robin and the grid is a multiple of 8, sized to the blocks that fit on the chip at once); it takes
// the next position x + 8 k of its XCD's part of the tile list from the counter ctr[x] until the
// list is exhausted, so heavy and light tiles balance dynamically.  The last block to finish
// (counter ctr[8]) clears the counters for the next launch.
// Waves per SIMD: at least 2 (without the bound the FP64 variant is allocated past 256 registers,
// 1 wave per SIMD); 3 for the FP32 step variant (168 registers, no spill; it needs 172 unbounded, so
// the FP64 collision would otherwise cost a third of its occupancy).  The residual variant, which
// runs on checked steps only, keeps 2 rather than spill.
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 && (MODE == kModeStep0 || MODE == kModeStep) ? 3 : 2))) void stage_kernel(const InstDesc* __restrict__ descs,
                                                         const TileRef* __restrict__ tiles, int ntiles,
                                                         int stage, unsigned* __restrict__ ctr)
{
    constexpr bool ANALYZE = MODE == kModeAnalyze;
    constexpr bool HAS_FN = MODE == kModeStep || MODE == kModeResid;  // stages 2 and 3 combine with f^n
    constexpr bool kDma = std::is_same<T, float>::value && !ANALYZE;  // windows prefetched through LDS
    // dynamic LDS: [union of (cell tables of the tile) and (moment reduction)] + boundary faces
    extern __shared__ __align__(16) unsigned char smem[];
    double(*lds_mom)[kRows][kTileCells] = reinterpret_cast<double(*)[kRows][kTileCells]>(smem);
    // the window prefetch buffers of the FP32 kernels: an LDS object of their own, so that the
    // compiler tells them apart from the cell tables (no wait for the prefetch before table reads)
    unsigned char* pfbuf = nullptr;
    if constexpr (kDma) {
        __shared__ __align__(16) unsigned char s_pf[(kThreads / 64) * kPfWave];
        pfbuf = s_pf;
    }
    double* const lds_sc = reinterpret_cast<double*>(smem);
    T* const lds_g = reinterpret_cast<T*>(smem + sizeof(double) * kNSc * kScSlot);
    __shared__ double lds_red[kThreads / 64][2];

    const int tid = threadIdx.x;
    const int row = tid / kTPR, strip = tid % kTPR;
    const int in_idx = ANALYZE ? 0 : (stage == 0 ? 0 : stage == 1 ? 1 : 2);
    const int out_idx = ANALYZE ? 0 : (stage == 0 ? 1 : stage == 1 ? 2 : 0);
    const double ca = stage == 1 ? 0.75 : stage == 2 ? (1.0 / 3.0) : 0.0;
    const double cb = stage == 1 ? 0.25 : stage == 2 ? (2.0 / 3.0) : 1.0;
    constexpr bool want_res = MODE == kModeResid;
    constexpr uint32_t es = sizeof(T);

    __shared__ int s_next;
    const int xcd = blockIdx.x % kXcds;
    for (;;) {
        __syncthreads();  // every thread has read the previous s_next
        if (tid == 0) s_next = xcd + kXcds * (int)atomicAdd(&ctr[xcd], 1u);
        __syncthreads();
        const int t = s_next;
        if (t >= ntiles) break;
        const TileRef tr = tiles[t];
        if (tr.inst < 0) continue;  // padding of the XCD-aware tile order (uniform per block)
        const InstDesc& D = descs[tr.inst];
        const int nx = D.nx, nv = D.nv, qx = D.qx, qy = D.qy, vpt = D.vpt;
        const int c0 = tr.ctile * kTileCells;
        const int s0 = c0 + strip * kStrip;
        const int seg = tr.group * kRows + row;
        const bool row_on = seg < D.nseg;
        const bool active = row_on && s0 < nx;
        const int hi = row_on ? seg / D.segs_per_line : 0;
        const int jc = seg - hi * D.segs_per_line;
        const double pxd = row_on ? D.px[hi] : 0.0;
        const T px = (T)pxd;
        const int vbase = hi * qy + jc * vpt;
        const uint32_t state_bytes = 2u * (uint32_t)nv * (uint32_t)nx * es;
        const __amdgpu_buffer_rsrc_t rin = make_rsrc(D.f[in_idx], state_bytes);
        const double nwl = D.dyn[DY_NWL], nwr = D.dyn[DY_NWR];
        const double Tw = D.Tw;
        // window offsets of the lane: cells s0-4.., s0.., s0+4.. (idle lanes read cells 0..3)
        const int sc = active ? s0 : 0;
        const bool last = s0 + kStrip == nx;
        const uint32_t oL = (uint32_t)(active && s0 != 0 ? s0 - 4 : sc) * es;
        const uint32_t oC = (uint32_t)sc * es;
        const uint32_t oR = (uint32_t)(active && !last ? s0 + 4 : sc) * es;
        const uint32_t rowstep = (uint32_t)nx * es;
        const uint32_t chi_off = (uint32_t)nv * rowstep;
        // offset of velocity vbase + k: the lane's rowoff plus the wave-uniform k rowstep
        const uint32_t rowoff = (uint32_t)vbase * rowstep;
        // this wave's prefetch buffer and the lane's LDS byte address in it
        unsigned char* const pf = pfbuf + __builtin_amdgcn_readfirstlane(tid / 64) * kPfWave;  // wave-uniform
        const uint32_t pf_la = (uint32_t)(uintptr_t)(lds_ptr)pf + (uint32_t)(tid % 64) * 16u;
        // the strip at cell 0: the left wall closure (full channel) or the mirrored ghosts (half channel)
        const bool first = s0 == 0 && !D.half, mirror = s0 == 0 && D.half;
        // rows of the mirrored velocities (-p_x, -p_y): the other sign of the half-range node, the
        // full-range node of opposite sign (nodes symmetric about 0, ascending)
        const int hmir = hi < qx ? hi + qx : hi - qx;
        const int jbase = vbase - hi * qy;  // j of the row's first velocity
        const __amdgpu_buffer_rsrc_t rfn = make_rsrc(D.f[0], state_bytes);
        // the prefetch of velocity k: windows, f^n (stages 2 and 3), and for the strip at cell 0 of
        // a half channel the mirrored cells in place of the left windows
        auto prefetch = [&](int k) {
            const uint32_t ks = (uint32_t)k * rowstep;
            dma16(rin, pf + 0 * kPfLoad, rowoff + oL, ks);
            dma16(rin, pf + 1 * kPfLoad, rowoff + oC, ks);
            dma16(rin, pf + 2 * kPfLoad, rowoff + oR, ks);
            dma16(rin, pf + 3 * kPfLoad, chi_off + rowoff + oL, ks);
            dma16(rin, pf + 4 * kPfLoad, chi_off + rowoff + oC, ks);
            dma16(rin, pf + 5 * kPfLoad, chi_off + rowoff + oR, ks);
            if constexpr (HAS_FN) {
                dma16(rfn, pf + 6 * kPfLoad, rowoff + oC, ks);
                dma16(rfn, pf + 7 * kPfLoad, chi_off + rowoff + oC, ks);
            }
            if (mirror) {
                const uint32_t moff = (uint32_t)(hmir * qy + (qy - 1 - (jbase + k))) * rowstep;
                dma16(rin, pf + 0 * kPfLoad, moff, 0u);
                dma16(rin, pf + 3 * kPfLoad, chi_off + moff, 0u);
            }
        };
        // the first velocity's loads travel while the cell tables are staged
        if constexpr (kDma)
            if (row_on) prefetch(0);
        // per-tile copies of p_y (all j) and of the wall populations of the tile's velocities
        double* const lds_py = reinterpret_cast<double*>(smem + cell_lds_bytes(qy, es));
        // wall equilibria g_x(0,T_w) g_y(-/+u_w,T_w) of the tile's velocities in the storage precision (the
        // wall populations they scale are stored in it): [left, right][row][k]
        T* const lds_gw = reinterpret_cast<T*>(lds_py + qy);

        if (!ANALYZE) {
            // stage the tile's cell tables: the FP64 scalars; 1/(J deta), g_y (all j) and g_x of each
            // row's node in the storage precision
            const __amdgpu_buffer_rsrc_t rsc = make_rsrc(D.sc, (uint32_t)kNSc * (uint32_t)nx * 8u);
            const __amdgpu_buffer_rsrc_t rg = make_rsrc(D.cell, (uint32_t)g_slots(qx, qy) * (uint32_t)nx * es);
            const int nsl = kNSc + g_lds_slots(qy);
            for (int ch = tid; ch < nsl * (kTileCells / 4); ch += kThreads) {
                const int slot = ch / (kTileCells / 4), q4 = ch % (kTileCells / 4);
                const int cell = c0 + 4 * q4;
                const uint32_t cc = (uint32_t)(cell < nx ? cell : 0);
                if (slot < kNSc) {
                    double v4[4];
                    bld4(rsc, ((uint32_t)slot * nx + cc) * 8u, v4);
#pragma unroll
                    for (int c = 0; c < 4; ++c) lds_sc[slot * kScSlot + c * kTPR + q4] = v4[c];
                } else {
                    const int gs = slot - kNSc;
                    int src;
                    if (gs == 0)
                        src = kGIjd;
                    else if (gs <= qy)
                        src = kGx0 + 2 * qx + (gs - 1);
                    else {
                        const int r = gs - 1 - qy, sg = tr.group * kRows + r;
                        src = kGx0 + (sg < D.nseg ? sg / D.segs_per_line : 0);
                    }
                    T v4[4];
                    bld4(rg, ((uint32_t)src * nx + cc) * es, v4);
#pragma unroll
                    for (int c = 0; c < 4; ++c) lds_g[gs * kLdsSlot + c * kTPR + q4] = v4[c];
                }
            }
            if constexpr (kDma) {
                for (int i = tid; i < qy; i += kThreads) lds_py[i] = D.py[i];
                for (int i = tid; i < kRows * vpt; i += kThreads) {
                    const int r = i / vpt, kk = i - r * vpt, sg = tr.group * kRows + r;
                    double gl = 0.0, gr = 0.0;
                    if (sg < D.nseg) {
                        const int h = sg / D.segs_per_line, vv = h * qy + (sg - h * D.segs_per_line) * vpt + kk;
                        gl = D.gw_l[vv];
                        gr = D.gw_r[vv];
                    }
                    lds_gw[i] = (T)gl;
                    lds_gw[kRows * vpt + i] = (T)gr;
                }
            }
            __syncthreads();
        }

        double acc[6][kStrip];
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int c = 0; c < kStrip; ++c) acc[a][c] = 0.0;
        double rnum = 0, rden = 0;

        if (row_on) {
            const __amdgpu_buffer_rsrc_t rout = make_rsrc(D.f[out_idx], state_bytes);
            // residual weights: J_s deta for ||f_old||, J_s deta (dt/dt_s)^2 for ||f_new - f_old|| / dt
            double jw[kStrip] = {0, 0, 0, 0}, jr[kStrip] = {0, 0, 0, 0};
            if (want_res && active)
#pragma unroll
                for (int c = 0; c < kStrip; ++c) {
                    jw[c] = D.jdeta[s0 + c];
                    jr[c] = D.jres[s0 + c];
                }
            double dtc[kStrip];  // time step of each cell (local time steps, or dt everywhere)
#pragma unroll
            for (int c = 0; c < kStrip; ++c) dtc[c] = ANALYZE ? 0.0 : D.dts[sc + c];
            uint32_t rkey = 0;
            if (!ANALYZE && D.rounding) {
                const uint32_t stepc = (uint32_t)D.dyn[DY_STEP];
                rkey = hash32(D.seed ^ hash32(stepc * 3u + (uint32_t)stage + 0x9e3779b9u));
            }
            const int rounding = ANALYZE ? 0 : D.rounding;
            if constexpr (kDma) {
                // the loads above have completed before the loop: inside it the memory counter also
                // counts the prefetch, and a wait for one of them would wait for the prefetch too
                __asm__ volatile("" ::"v"(dtc[0]), "v"(dtc[1]), "v"(dtc[2]), "v"(dtc[3]), "v"(px), "v"(pxd));
                if constexpr (want_res)
                    __asm__ volatile("" ::"v"(jw[0]), "v"(jw[1]), "v"(jw[2]), "v"(jw[3]), "v"(jr[0]), "v"(jr[1]),
                                     "v"(jr[2]), "v"(jr[3]));
            }
            uint32_t kstep = 0;
            for (int k = 0; k < vpt; ++k, kstep += rowstep) {
                Win<T> P, X;
                T fnp[4] = {T(0), T(0), T(0), T(0)}, fnc[4] = {T(0), T(0), T(0), T(0)};
                const int v = vbase + k;
                const int j = v - hi * qy;
                double pyd, gl = 0.0, gr = 0.0;
                if constexpr (kDma) {
                    // velocity k is in the buffer once every operation but the last two (the previous
                    // velocity's output stores) has retired
                    f4v t[kPfSlots];
                    constexpr int nslot = HAS_FN ? 8 : 6;
                    if (k == 0)
                        read_slots<0, nslot>(pf_la, t);
                    else
                        read_slots<2, nslot>(pf_la, t);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        P.w[c] = t[0][c];
                        X.w[c] = t[3][c];
                        P.w[4 + c] = t[1][c];
                        P.w[8 + c] = t[2][c];
                        X.w[4 + c] = t[4][c];
                        X.w[8 + c] = t[5][c];
                        if constexpr (HAS_FN) {
                            fnp[c] = t[6][c];
                            fnc[c] = t[7][c];
                        }
                    }
                    if (mirror)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            // point symmetry of Sec. II about x = 0 (half channel, strip at cell 0): ghost
                            // cells -1..-4 of (p_x, p_y) hold the values of (-p_x, -p_y) in cells 0..3
                            P.w[c] = t[0][3 - c];
                            X.w[c] = t[3][3 - c];
                        }
                    pyd = lds_py[j];
                    gl = lds_gw[row * vpt + k];
                    gr = lds_gw[(kRows + row) * vpt + k];
                    // the next velocity's loads (none after the last: the epilogue drains the counter)
                    if (k + 1 < vpt) prefetch(k + 1);
                } else {
                    T tmp[4];
                    bld4(rin, rowoff + oL, tmp, kstep);
#pragma unroll
                    for (int c = 0; c < 4; ++c) P.w[c] = tmp[c];
                    bld4(rin, rowoff + oC, tmp, kstep);
#pragma unroll
                    for (int c = 0; c < 4; ++c) P.w[4 + c] = tmp[c];
                    bld4(rin, rowoff + oR, tmp, kstep);
#pragma unroll
                    for (int c = 0; c < 4; ++c) P.w[8 + c] = tmp[c];
                    bld4(rin, chi_off + rowoff + oL, tmp, kstep);
#pragma unroll
                    for (int c = 0; c < 4; ++c) X.w[c] = tmp[c];
                    bld4(rin, chi_off + rowoff + oC, tmp, kstep);
#pragma unroll
                    for (int c = 0; c < 4; ++c) X.w[4 + c] = tmp[c];
                    bld4(rin, chi_off + rowoff + oR, tmp, kstep);
#pragma unroll
                    for (int c = 0; c < 4; ++c) X.w[8 + c] = tmp[c];
                    pyd = D.py[j];
                    if (!ANALYZE && mirror) {
                        // point symmetry of Sec. II about x = 0: ghost cells -1..-4 of (p_x, p_y) hold
                        // the values of (-p_x, -p_y) in cells 0..3
                        const uint32_t moff = (uint32_t)(hmir * qy + (qy - 1 - j)) * rowstep;
                        bld4(rin, moff, tmp);
#pragma unroll
                        for (int c = 0; c < 4; ++c) P.w[3 - c] = tmp[c];
                        bld4(rin, chi_off + moff, tmp);
#pragma unroll
                        for (int c = 0; c < 4; ++c) X.w[3 - c] = tmp[c];
                    }
                    if constexpr (HAS_FN) {
                        bld4(rfn, rowoff + oC, fnp, kstep);
                        bld4(rfn, chi_off + rowoff + oC, fnc, kstep);
                    }
                    if (!ANALYZE && first) gl = D.gw_l[v];
                    if (!ANALYZE && last) gr = D.gw_r[v];
                }
                // wall populations (eq. diffuse) of this velocity: only the strips next to a wall use them
                T phiwl = T(0), chiwl = T(0), phiwr = T(0), chiwr = T(0);
                if (!ANALYZE && first) {
                    phiwl = (T)(nwl * gl);
                    chiwl = (T)(Tw * nwl * gl);
                }
                if (!ANALYZE && last) {
                    phiwr = (T)(nwr * gr);
                    chiwr = (T)(Tw * nwr * gr);
                }
                T op[kStrip], oc[kStrip];
                if (ANALYZE) {
#pragma unroll
                    for (int c = 0; c < kStrip; ++c) {
                        op[c] = P.w[4 + c];
                        oc[c] = X.w[4 + c];
                    }
                } else {
                    // ghosts: entering directions take the wall populations, leaving ones the
                    // quadratic extrapolation of the three cells next to the wall.  A leaving face at
                    // a wall is then the window's own face: its five cells and its operations are
                    // those of wall_face_left / wall_face_right, so it has the same bits as the wall
                    // fluxes the per-cell kernel forms.  An entering face is the wall population.
                    T Fp[5], Fc[5];
                    if (px > T(0)) {
                        if (first) {
                            P.w[1] = P.w[2] = P.w[3] = phiwl;
                            X.w[1] = X.w[2] = X.w[3] = chiwl;
                        }
                        if (last) {
                            P.w[8] = ext_p3(P.w[5], P.w[6], P.w[7]);
                            P.w[9] = ext_p4(P.w[5], P.w[6], P.w[7]);
                            X.w[8] = ext_p3(X.w[5], X.w[6], X.w[7]);
                            X.w[9] = ext_p4(X.w[5], X.w[6], X.w[7]);
                        }
                        P.faces_pos(Fp);
                        X.faces_pos(Fc);
                        if (first) {
                            Fp[0] = phiwl;
                            Fc[0] = chiwl;
                        }
                    } else {
                        if (first) {
                            P.w[3] = ext_m1(P.w[4], P.w[5], P.w[6]);
                            P.w[2] = ext_m2(P.w[4], P.w[5], P.w[6]);
                            X.w[3] = ext_m1(X.w[4], X.w[5], X.w[6]);
                            X.w[2] = ext_m2(X.w[4], X.w[5], X.w[6]);
                        }
                        if (last) {
                            P.w[8] = P.w[9] = P.w[10] = phiwr;
                            X.w[8] = X.w[9] = X.w[10] = chiwr;
                        }
                        P.faces_neg(Fp);
                        X.faces_neg(Fc);
                        if (last) {
                            Fp[4] = phiwr;
                            Fc[4] = chiwr;
                        }
                    }
                    if constexpr (kDma && HAS_FN) {
                        // the previous stage's values are first needed by the combine: their loads
                        // overlap the face computation
#pragma unroll
                        for (int c = 0; c < kStrip; ++c)
                            __asm__ volatile("" : "+v"(fnp[c]), "+v"(fnc[c]) : "v"(Fp[kStrip]), "v"(Fc[kStrip]));
                    }
                    uint32_t rbits[kStrip] = {0, 0, 0, 0};
                    if (rounding) {
                        const uint32_t base = rkey ^ ((uint32_t)v * 0x85ebca6bu) ^ ((uint32_t)s0 * 0xc2b2ae35u);
#pragma unroll
                        for (int c = 0; c < kStrip; ++c) rbits[c] = c == 0 ? hash32(base) : weyl32(rbits[c - 1]);
                    }
                    int lcol = strip;
                    // an opaque column index keeps the compiler from hoisting the per-cell terms out of
                    // the velocity loop into registers (they stay in LDS; occupancy 3 instead of 2)
                    __asm__ volatile("" : "+v"(lcol));
                    const double* Ls = lds_sc + lcol;
                    const T* Lg = lds_g + lcol;
#pragma unroll
                    for (int c = 0; c < kStrip; ++c) {
                        const T p = P.w[4 + c], x = X.w[4 + c];
                        const double ux = Ls[SC_UX * kScSlot + c * kTPR], uy = Ls[SC_UY * kScSlot + c * kTPR];
                        const double Tt = Ls[SC_T * kScSlot + c * kTPR], itau = Ls[SC_INVTAU * kScSlot + c * kTPR];
                        const double S8 = Ls[SC_S8 * kScSlot + c * kTPR], S4 = Ls[SC_S4 * kScSlot + c * kTPR];
                        const double A5 = Ls[SC_AS5T * kScSlot + c * kTPR];
                        const double qxv = Ls[SC_QX * kScSlot + c * kTPR], qyv = Ls[SC_QY * kScSlot + c * kTPR];
                        const T ijd = Lg[kGIjd * kLdsSlot + c * kTPR];
                        const T gy = Lg[(1 + j) * kLdsSlot + c * kTPR];
                        const T gx = Lg[(1 + qy + row) * kLdsSlot + c * kTPR];
                        // reduced Shakhov collision, Sec. II, in FP64: with xi = p - u, the targets
                        // phi_eq (1 + S_phi) and chi_eq (1 + S_chi) = T phi_eq (1 + S_chi), where
                        // S_phi = (q.xi) (A xi^2/(5T) - 0.8 A), S_chi = (q.xi) (A xi^2/(5T) - 0.4 A); with
                        // W = phi_eq (q.xi) and V = phi_eq + W A xi^2/(5T) they are V - 0.8 A W and
                        // T (V - 0.4 A W) (the product of the truncated equilibria is exact in FP64)
                        const double xx = pxd - ux, xy = pyd - uy;
                        const double x2 = xx * xx + xy * xy;
                        const double qxi = qxv * xx + qyv * xy;
                        const double feq = (double)gx * (double)gy;
                        const double W = feq * qxi;
                        const double V = fma(W, A5 * x2, feq);
                        const double tp = fma(-W, S8, V);
                        const double tc = Tt * fma(-W, S4, V);
                        // x-advection in the storage precision: -p_x (F_{s+1/2} - F_{s-1/2}) / (J_s deta)
                        const T mpi = -px * ijd;
                        const T ap = (Fp[c + 1] - Fp[c]) * mpi;
                        const T ax = (Fc[c + 1] - Fc[c]) * mpi;
                        const double Lp = (double)ap + (tp - (double)p) * itau;
                        const double Lx = (double)ax + (tc - (double)x) * itau;
                        // SSP-RK3 stage: out = a f^n + b (f_in + dt L(f_in)), combined in FP64 (a = 0, b = 1
                        // in the first stage, which reads no f^n)
                        double fnpd = 0.0, fncd = 0.0, ope, oce;
                        if constexpr (HAS_FN) {
                            fnpd = (double)fnp[c];
                            fncd = (double)fnc[c];
                            ope = ca * fnpd + cb * ((double)p + dtc[c] * Lp);
                            oce = ca * fncd + cb * ((double)x + dtc[c] * Lx);
                        } else {
                            ope = (double)p + dtc[c] * Lp;
                            oce = (double)x + dtc[c] * Lx;
                        }
                        op[c] = store_round<T>(ope, rounding, rbits[c]);
                        oc[c] = store_round<T>(oce, rounding, rbits[c] >> 16);
                        if (want_res) {
                            const double dp = ope - fnpd, dc = oce - fncd;
                            rnum += jr[c] * (dp * dp + dc * dc);
                            rden += jw[c] * (fnpd * fnpd + fncd * fncd);
                        }
                    }
                    if (active) {
                        bst4(rout, rowoff + oC, op, kstep);
                        bst4(rout, chi_off + rowoff + oC, oc, kstep);
                    }
                }
                if (active) {
                    // moments of the output (FP64): sums over this row's j of phi p_y^a and chi p_y^b
                    const double py2 = pyd * pyd, py3 = py2 * pyd;
#pragma unroll
                    for (int c = 0; c < kStrip; ++c) {
                        const double o = (double)op[c], x = (double)oc[c];
                        acc[0][c] += o;
                        acc[1][c] += pyd * o;
                        acc[2][c] += py2 * o;
                        acc[3][c] += py3 * o;
                        acc[4][c] += x;
                        acc[5][c] += pyd * x;
                    }
                }
            }
        }
        // the last prefetch has landed before its LDS becomes part of the moment sums
        if constexpr (kDma) vm_drain();
        if (!ANALYZE) __syncthreads();  // the LDS region switches from cell tables to moment sums

        // ---- moments: combine the row sums with the powers of p_x, reduce rows in LDS ----------
        double m11[kNMom][kStrip];
        {
            const double px1 = pxd, px2 = pxd * pxd, px3 = px2 * pxd;
#pragma unroll
            for (int c = 0; c < kStrip; ++c) {
                const double A0 = acc[0][c], A1 = acc[1][c], A2 = acc[2][c], A3 = acc[3][c];
                const double B0 = acc[4][c], B1 = acc[5][c];
                m11[0][c] = A0;
                m11[1][c] = px1 * A0;
                m11[2][c] = A1;
                m11[3][c] = px2 * A0;
                m11[4][c] = px1 * A1;
                m11[5][c] = A2;
                m11[6][c] = px3 * A0 + px1 * A2;
                m11[7][c] = px2 * A1 + A3;
                m11[8][c] = B0;
                m11[9][c] = px1 * B0;
                m11[10][c] = B1;
            }
        }
        // the FP32 step kernels reduce in the drained prefetch buffers (4 moments per pass, like FP64)
        constexpr int kMpp = kDma ? kMomPerPass : moments_per_pass(sizeof(T));
        static_assert(!kDma || sizeof(double) * kMomPerPass * kRows * kTileCells <= (kThreads / 64) * kPfWave,
                      "moment passes fit the prefetch buffers");
        double(*const lds_red_mom)[kRows][kTileCells] =
            kDma ? reinterpret_cast<double(*)[kRows][kTileCells]>(pfbuf) : lds_mom;
#pragma unroll
        for (int pass = 0; pass < (kNMom + kMpp - 1) / kMpp; ++pass) {
#pragma unroll
            for (int mm = 0; mm < kMpp; ++mm) {
                const int m = pass * kMpp + mm;
                if (m < kNMom) {
                    // position c * 16 + strip: the 16 lanes of a row write 16 consecutive words
#pragma unroll
                    for (int c = 0; c < kStrip; ++c) lds_red_mom[mm][row][c * kTPR + strip] = m11[m][c];
                }
            }
            __syncthreads();
            {
                // lane l of the reading wave takes position l: cell 4 (l % 16) + l / 16 of the tile
                const int mm = tid / kTileCells, pos = tid % kTileCells;
                const int m = pass * kMpp + mm;
                const int cellx = c0 + (pos % kTPR) * kStrip + pos / kTPR;
                if (mm < kMpp && m < kNMom && cellx < nx) {
                    double s = 0.0;
#pragma unroll
                    for (int r = 0; r < kRows; ++r) s += lds_red_mom[mm][r][pos];
                    D.mom_part[((size_t)tr.group * kNMom + m) * nx + cellx] = s;
                }
            }
            __syncthreads();
        }

        // ---- residual partials: block sums in a fixed order ------------------------------------
        if (want_res) {
            double vals[2] = {rnum, rden};
            const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double s = wave_sum(vals[q]);
                if (lane == 0) lds_red[wave][q] = s;
            }
            __syncthreads();
            if (tid == 0) {
                for (int q = 0; q < 2; ++q) {
                    double s = 0.0;
                    for (int w = 0; w < kThreads / 64; ++w) s += lds_red[w][q];
                    D.res_part[tr.tile_id * 2 + q] = s;
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        // no block touches the counters after its own increment of ctr[kXcds]: the last one resets
        if (atomicAdd(&ctr[kXcds], 1u) == gridDim.x - 1)
            for (int x = 0; x <= kXcds; ++x) ctr[x] = 0u;
    }
}

// ---- per-cell kernel --------------------------------------------------------------------------
// A block of kCellThreads threads serves kCellThreads / L cells with L = cell_lanes lanes per cell
// (1 to 16; 2 unless the plan says otherwise): the lanes of a cell split the sums of the moment
// partials over velocity groups, the auxiliary-rule sums of g_x and the output nodes of g_x and
// g_y, and combine their partial sums by an xor butterfly (identical bits in every lane).  Two more
// blocks per instance each reduce the leaving fluxes through one wall, beside the cell blocks.

// leaving fluxes through one wall (eq. diffuse_nw): block-wide sums over the leaving directions of
// p_x F and p_x p_y F, F the wall face value of the current state; fixed-order reduction
template <typename T>
__device__ void wall_sums(const InstDesc& D, const T* f, bool right, double& flux, double& mom)
{
    __shared__ double red[kCellThreads / 64][2];
    const int nx = D.nx, qx = D.qx, qy = D.qy, half = qx * qy;
    double a = 0.0, b = 0.0;
    for (int u = threadIdx.x; u < half; u += blockDim.x) {
        const int v = right ? u : half + u;  // right wall: p_x > 0 leave; left wall: p_x < 0 leave
        const T* r = f + (size_t)v * nx;
        const T F = right ? wall_face_right(r[nx - 3], r[nx - 2], r[nx - 1]) : wall_face_left(r[0], r[1], r[2]);
        const double pxv = D.px[v / qy], pyv = D.py[v % qy];
        a += pxv * (double)F;
        b += pxv * pyv * (double)F;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[wave][0] = a;
        red[wave][1] = b;
    }
    __syncthreads();
    flux = 0.0;
    mom = 0.0;
    for (int w = 0; w < kCellThreads / 64; ++w) {
        flux += red[w][0];
        mom += red[w][1];
    }
    __syncthreads();  // red may be reused by a second call in the same block
}

// the left wall of the current state (eq. diffuse_nw: n_w and the momentum flux; none in the half
// channel), and the count of a completed step; block-wide
template <typename T>
__device__ __forceinline__ void wall_left(const InstDesc& D, const T* fcur, int flags)
{
    if (!D.half) {
        double fl, ml;
        wall_sums<T>(D, fcur, false, fl, ml);
        if (threadIdx.x == 0) {
            const double nwl = -fl / D.den_l;
            D.dyn[DY_NWL] = nwl;
            D.dyn[DY_SHEAR_L] = ml + nwl * D.mom_l;
        }
    }
    if (threadIdx.x == 0 && (flags & FLAG_STEP_DONE)) {
        D.dyn[DY_STEP] += 1.0;
        if (D.dyn[DY_AVG_ON] != 0.0) D.dyn[DY_AVG_STEPS] += 1.0;
    }
}

// the right wall of the current state; block-wide
template <typename T>
__device__ __forceinline__ void wall_right(const InstDesc& D, const T* fcur)
{
    double fr, mr;
    wall_sums<T>(D, fcur, true, fr, mr);
    if (threadIdx.x == 0) {
        const double nwr = -fr / D.den_r;
        D.dyn[DY_NWR] = nwr;
        D.dyn[DY_SHEAR_R] = mr + nwr * D.mom_r;
    }
}

// sums over the lanes of a cell (lanes = 1, 2, 4, 8 or 16 consecutive lanes, aligned) of the N
// values x and the M values y: a butterfly whose step s adds the partner's value, identical in every
// lane afterwards.  The partners come from DPP patterns inside a 16-lane row (quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror): after the steps before it, every lane of a group
// of 2^s holds the same value, so these pair each group with the neighbouring one exactly as
// lane ^ 2^s would, and the sums (and their bits) are those of the xor butterfly, without a trip
// through LDS.  One uniform branch per step covers every value.
template <int N, int M = 0>
__device__ __forceinline__ void lane_sums(double (&x)[N], double (&y)[M > 0 ? M : 1], int lanes)
{
    auto step = [&](auto ctrl) {
        constexpr int C = decltype(ctrl)::value;
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] += dpp_partner<C>(x[i]);
#pragma unroll
        for (int i = 0; i < M; ++i) y[i] += dpp_partner<C>(y[i]);
    };
    if (lanes > 1) step(std::integral_constant<int, 0xB1>());
    if (lanes > 2) step(std::integral_constant<int, 0x4E>());
    if (lanes > 4) step(std::integral_constant<int, 0x141>());
    if (lanes > 8) step(std::integral_constant<int, 0x140>());
}

// eq. (gx) as the projection of g/omega on h_0..h_{NB-1} (rows beyond N_x are zero) with the
// auxiliary rule: lane q of the cell takes nodes k = q, q + L, ...; three nodes per iteration (up to
// 8 rows) or two (up to 11) keep that many independent exponential chains in flight (one node per
// iteration for the largest row count, whose accumulators already fill the register budget).  Partial
// sums in k order, then an xor butterfly.
// The rule is scaled to T_w (nodes Z of the weight exp(-p^2/(2 T_w))), on which the integrand is
// exp(Z^2 (T/T_w - 1)/(2T) + Z u/T - u^2/(2T))/sqrt(T) h_l(Z).
template <int NB>
__device__ __forceinline__ void gx_project(int q, int LN, double Tm, double Tw, double ux, int K,
                                           const double* s_az, const double* s_aw, const double* s_hZ,
                                           double (&Ip)[NB], double (&Im)[NB])
{
#pragma unroll
    for (int l = 0; l < NB; ++l) Ip[l] = Im[l] = 0.0;
    const double inv2T = 0.5 / Tm;
    const double rsT = 1.0 / sqrt(Tm);
    const double c0 = ((Tm - Tw) / Tw) * inv2T, c1 = ux * (2.0 * inv2T), c2 = ux * ux * inv2T;
    int k = q;
    for (; NB <= 8 && k + 2 * LN < K; k += 3 * LN) {
        double ep[3], em[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const double Z = s_az[k + u * LN];
            const double a = Z * Z * c0 - c2, bb = Z * c1;
            const double wk = s_aw[k + u * LN] * rsT;
            ep[u] = wk * exp_cw(a + bb);
            em[u] = wk * exp_cw(a - bb);
        }
#pragma unroll
        for (int l = 0; l < NB; ++l)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const double h = s_hZ[l * K + k + u * LN];
                Ip[l] += ep[u] * h;
                Im[l] += em[u] * h;
            }
    }
    for (; NB <= 11 && k + LN < K; k += 2 * LN) {
        const double Z0 = s_az[k], Z1 = s_az[k + LN];
        const double a0 = Z0 * Z0 * c0 - c2, a1 = Z1 * Z1 * c0 - c2;
        const double b0 = Z0 * c1, b1 = Z1 * c1;
        const double w0 = s_aw[k] * rsT, w1 = s_aw[k + LN] * rsT;
        const double ep0 = w0 * exp_cw(a0 + b0), ep1 = w1 * exp_cw(a1 + b1);
        const double em0 = w0 * exp_cw(a0 - b0), em1 = w1 * exp_cw(a1 - b1);
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            const double h0 = s_hZ[l * K + k], h1 = s_hZ[l * K + k + LN];
            Ip[l] += ep0 * h0;
            Im[l] += em0 * h0;
            Ip[l] += ep1 * h1;
            Im[l] += em1 * h1;
        }
    }
    for (; k < K; k += LN) {
        const double Z = s_az[k];
        const double a = Z * Z * c0 - c2, bb = Z * c1;
        const double wk = s_aw[k] * rsT;
        const double ep = wk * exp_cw(a + bb), em = wk * exp_cw(a - bb);
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            const double h = s_hZ[l * K + k];
            Ip[l] += ep * h;
            Im[l] += em * h;
        }
    }
    // rows beyond N_x hold zeros in every lane: summing them leaves them zero
    lane_sums<NB, NB>(Ip, Im, LN);
}

// g_x at the 2 Q_x nodes from the projections: n w_i sum_l I_l h_l(z_i); small: the 24-node
// auxiliary rule (ktab at s_az2), else the 48-node one.  With 16 lanes per cell the 24 nodes would
// split unevenly over the lanes (pairs on 8 of them, single nodes on the others: both paths in every
// wave, no faster than the 48-node split), so such plans keep the 48-node rule.
template <typename T, int NB, typename CP>
__device__ __forceinline__ void gx_nodes(int q, int LN, double n, double Tm, double Tw, double ux, bool small, bool on,
                                         int s, int nx, int qxn, const double* s_wx, const double* s_az,
                                         const double* s_aw, const double* s_hZ, const double* s_az2,
                                         const double* s_hz, CP cell)
{
    double Ip[NB], Im[NB];
    if (small)
        gx_project<NB>(q, LN, Tm, Tw, ux, kAux2, s_az2, s_az2 + kAux2, s_az2 + 2 * kAux2, Ip, Im);
    else
        gx_project<NB>(q, LN, Tm, Tw, ux, kAux, s_az, s_aw, s_hZ, Ip, Im);
    for (int i = q; i < qxn; i += LN) {
        double ap = 0.0, am = 0.0;
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            const double hz = s_hz[l * qxn + i];
            ap += Ip[l] * hz;
            am += Im[l] * hz;
        }
        const double nw = n * s_wx[i];
        if (on) {
            cell[(kGx0 + i) * nx + s] = (T)(nw * ap);
            cell[(kGx0 + qxn + i) * nx + s] = (T)(nw * am);
        }
    }
}

// eq. (gy): c_l = coefficient of t^l in exp(u t + (T-1) t^2/2), l c_l = u c_{l-1} + (T-1) c_{l-2};
// NB rows of the He table, zero beyond N_y
template <typename T, int NB, typename CP>
__device__ __forceinline__ void gy_nodes(int q, int LN, int nyo, double uy, double Tm, bool on, int s, int nx,
                                         int qxn, int nqy, const double* s_wy, const double* s_he, CP cell)
{
    const double tm1 = Tm - 1.0;
    double cl[NB];
    cl[0] = 1.0;
    cl[1] = uy;
#pragma unroll
    for (int l = 2; l < NB; ++l) cl[l] = (uy * cl[l - 1] + tm1 * cl[l - 2]) * (1.0 / l);
#pragma unroll
    for (int l = 2; l < NB; ++l) cl[l] = l <= nyo ? cl[l] : 0.0;
    for (int j = q; j < nqy; j += LN) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < NB; ++l) acc += cl[l] * s_he[l * nqy + j];
        if (on) cell[(kGx0 + 2 * qxn + j) * nx + s] = (T)(s_wy[j] * acc);
    }
}

// the same for orders beyond the unrolled buckets: the recurrence runs once per output node
template <typename T, typename CP>
__device__ __forceinline__ void gy_nodes_long(int q, int LN, int nyo, double uy, double Tm, bool on, int s, int nx,
                                              int qxn, int nqy, const double* s_wy, const double* s_he, CP cell)
{
    const double tm1 = Tm - 1.0;
    for (int j = q; j < nqy; j += LN) {
        double c2 = 1.0, c1 = uy;
        double acc = s_he[j] + uy * s_he[nqy + j];
        for (int l = 2; l <= nyo; ++l) {
            const double c = (uy * c1 + tm1 * c2) / l;
            acc += c * s_he[l * nqy + j];
            c2 = c1;
            c1 = c;
        }
        if (on) cell[(kGx0 + 2 * qxn + j) * nx + s] = (T)(s_wy[j] * acc);
    }
}

// The per-cell part of the per-cell kernel: from the raw moment sums R of cell s (the partial sums of
// the cell's LN lanes, lane q) to the FP64 scalars sc[slot * nx + s] and the storage-precision table
// cell[slot * nx + s] of the next stage, and with FLAG_STEP_DONE / FLAG_FIELDS the fields, the running
// averages and the range flag.  Shared by the per-cell kernel (global tables) and the small-case kernel
// (tables in LDS, same layout).
// SMALLB: only the unrolled buckets of expansion orders up to N_x = 10, N_y = 11 (the small-case path
// admits no others), which keeps its register use down.  avg: whether the running averages are on
// (read by the caller)
template <typename T, bool SMALLB = false>
__device__ __forceinline__ void cell_tables(const InstDesc& D, double (&R)[kNMom], int q, int LN, int s, bool on,
                                            int flags, double* sc, T* cell, const double* ktab, const CellLds& lay,
                                            int avg)
{
    const int nx = D.nx;
    const int qxn = D.qx, nqy = D.qy, nyo = D.nyo, nxb = D.nxb, nyb = D.nyb;
    const double* s_wx = ktab + lay.wx;
    const double* s_wy = ktab + lay.wy;
    const double* s_az = ktab + lay.az;
    const double* s_aw = ktab + lay.aw;
    const double* s_hZ = ktab + lay.hZ;
    const double* s_hz = ktab + lay.hz;
    const double* s_he = ktab + lay.he;
    const double* s_az2 = ktab + lay.az2;
    // the tiled path's tables are global memory, the small-case path's LDS
    const auto scp = [&]() {
        if constexpr (SMALLB) return sc; else return gmem(sc);
    }();
    const auto cellp = [&]() {
        if constexpr (SMALLB) return cell; else return gmem(cell);
    }();
    {
        double none[1];
        lane_sums<kNMom>(R, none, LN);
    }

    // moments of Sec. II from the raw sums (shift to the peculiar velocity xi = p - u)
    const double n = R[0];
    const double ux = R[1] / n, uy = R[2] / n;
    const double pxx = R[3] - n * ux * ux;
    const double pxy = R[4] - n * ux * uy;
    const double pyy = R[5] - n * uy * uy;
    const double tzz = R[8];
    const double Tm = (pxx + pyy + tzz) / (3.0 * n);
    const double u2 = ux * ux + uy * uy;
    const double b = R[3] + R[5];
    const double c0 = ux * R[1] + uy * R[2];
    const double cx = ux * R[3] + uy * R[4];
    const double cy = ux * R[4] + uy * R[5];
    const double qx = 0.5 * (R[6] - ux * b - 2.0 * cx + 2.0 * ux * c0 + u2 * (R[1] - ux * R[0]) + R[9] - ux * R[8]);
    const double qy = 0.5 * (R[7] - uy * b - 2.0 * cy + 2.0 * uy * c0 + u2 * (R[2] - uy * R[0]) + R[10] - uy * R[8]);

    // eq. (tau) with mu ~ T^omega (eq. mu) or the tabulated law; Shakhov prefactor (1 - Pr)/(n K_B^2 T^2).
    // Every lane of the cell evaluates them (the same value): outside a one-lane branch the chain overlaps
    // the projection below instead of preceding it.
    double invtau, pr = D.Pr;
    if (D.ntab > 0) {
        // tabulated law, eqs. (mun) and (interp): 1/tau = tau_pref n (T/T_w) mu(T_w)/mu(T)
        double mu;
        visc_lookup(D.vT, D.vMu, D.vOm, D.vPr, D.ntab, Tm, &mu, &pr);
        invtau = D.tau_pref * n * (Tm / D.Tw) * (D.mu_w / mu);
    } else {
        // (T/T_w)^(1-omega) as an exponential of a logarithm: about half the instructions of pow, and
        // (T/T_w near 1, |1-omega| <= 1) within a few units in the last place of it
        invtau = D.tau_pref * n * exp_cw(D.visc_y * log(Tm * D.inv_Tw));
    }
    if (D.collisionless) invtau = 0.0;
    const double As = (1.0 - pr) / (n * Tm * Tm);
    const double As5T = As / (5.0 * Tm);

    if (on && q == 0) {
        if (flags & (FLAG_STEP_DONE | FLAG_FIELDS)) {
            const gptr<double> F = gmem(D.fields);
            F[F_N * nx + s] = n;
            F[F_UX * nx + s] = ux;
            F[F_UY * nx + s] = uy;
            F[F_T * nx + s] = Tm;
            F[F_PXX * nx + s] = pxx;
            F[F_PXY * nx + s] = pxy;
            F[F_PYY * nx + s] = pyy;
            F[F_TZZ * nx + s] = tzz;
            F[F_QX * nx + s] = qx;
            F[F_QY * nx + s] = qy;
        }
        scp[SC_UX * nx + s] = ux;
        scp[SC_UY * nx + s] = uy;
        scp[SC_T * nx + s] = Tm;
        scp[SC_INVTAU * nx + s] = invtau;
        scp[SC_S8 * nx + s] = 0.8 * As;
        scp[SC_S4 * nx + s] = 0.4 * As;
        scp[SC_AS5T * nx + s] = As5T;
        scp[SC_QX * nx + s] = qx;
        scp[SC_QY * nx + s] = qy;
        if constexpr (!SMALLB) cellp[kGIjd * nx + s] = (T)D.inv_jdeta[s];  // the small path fills it once
        // the band in which the projection of eq. (gx) is verified (a finite state outside it is
        // flagged; non-finite values are caught by the residual check)
        if (Tm < D.band_tlo || Tm > D.band_thi || fabs(ux) > D.band_u) gmem(D.dyn)[DY_RANGE] = 1.0;
        if ((flags & FLAG_STEP_DONE) && avg) {
            // running sums of the fields at the end of every step (time averages, hrlb_average_*)
            const gptr<double> A = gmem(D.avg);
            A[F_N * nx + s] += n;
            A[F_UX * nx + s] += ux;
            A[F_UY * nx + s] += uy;
            A[F_T * nx + s] += Tm;
            A[F_PXX * nx + s] += pxx;
            A[F_PXY * nx + s] += pxy;
            A[F_PYY * nx + s] += pyy;
            A[F_TZZ * nx + s] += tzz;
            A[F_QX * nx + s] += qx;
            A[F_QY * nx + s] += qy;
        }
    }

    // g_x (eq. gx) and g_y (eq. gy) with the loops over the expansion order unrolled for the case's
    // padded row count (uniform over the block); the 24-node auxiliary rule (ktab at s_az2) where it is
    // as accurate as the 48-node one (the same choice in every lane of a cell)
    const bool use2 = uses_aux2(LN) && Tm >= D.aux2_tlo && Tm <= D.aux2_thi && fabs(ux) <= D.aux2_u;
    switch (nxb) {
        case 4: gx_nodes<T, 4>(q, LN, n, Tm, D.Tw, ux, use2, on, s, nx, qxn, s_wx, s_az, s_aw, s_hZ, s_az2, s_hz, cellp); break;
        case 8: gx_nodes<T, 8>(q, LN, n, Tm, D.Tw, ux, use2, on, s, nx, qxn, s_wx, s_az, s_aw, s_hZ, s_az2, s_hz, cellp); break;
        case 11: gx_nodes<T, 11>(q, LN, n, Tm, D.Tw, ux, use2, on, s, nx, qxn, s_wx, s_az, s_aw, s_hZ, s_az2, s_hz, cellp); break;
        default:
            if constexpr (!SMALLB)
                gx_nodes<T, 17>(q, LN, n, Tm, D.Tw, ux, use2, on, s, nx, qxn, s_wx, s_az, s_aw, s_hZ, s_az2, s_hz, cellp);
            break;
    }
    if constexpr (SMALLB) {
        switch (nyb) {
            case 4: gy_nodes<T, 4>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
            case 8: gy_nodes<T, 8>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
            default: gy_nodes<T, 12>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        }
        return;
    }
    switch (nyb) {
        case 4: gy_nodes<T, 4>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        case 8: gy_nodes<T, 8>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        case 12: gy_nodes<T, 12>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        case 16: gy_nodes<T, 16>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        case 20: gy_nodes<T, 20>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        case 32: gy_nodes<T, 32>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
        default: gy_nodes_long<T>(q, LN, nyo, uy, Tm, on, s, nx, qxn, nqy, s_wy, s_he, cellp); break;
    }
}

// at most 128 registers: 4 waves per SIMD (the largest projection bucket spills a few words)
template <typename T>
__global__ __launch_bounds__(kCellThreads) __attribute__((amdgpu_waves_per_eu(4))) void cell_kernel(const InstDesc* __restrict__ descs,
                                                            const CellRef* __restrict__ cells, int buf, int flags)
{
    extern __shared__ double ktab[];
    const CellRef cr = cells[blockIdx.x];
    const InstDesc& D = descs[cr.inst];
    const int nx = D.nx;
    const T* fcur = (const T*)D.f[buf];
    if (cr.cell0 < 0) {  // a wall block (uniform per block)
        if (cr.cell0 == kWallLeft)
            wall_left<T>(D, fcur, flags);
        else
            wall_right<T>(D, fcur);
        return;
    }
    const int LN = D.cell_lanes;
    const int q = threadIdx.x & (LN - 1);
    const int s = cr.cell0 + threadIdx.x / LN;
    const bool on = s < nx;
    const int sc = on ? s : 0;
    // whether the running averages are on (read only at the end of a step), issued with the loads below
    const int avg = (flags & FLAG_STEP_DONE) ? (D.dyn[DY_AVG_ON] != 0.0) : 0;

    // moment partials of this cell: lane q sums the velocity groups g = q, q + L, ... (issued before
    // the table staging so that their latency overlaps it)
    double R[kNMom];
#pragma unroll
    for (int m = 0; m < kNMom; ++m) R[m] = 0.0;
    for (int g = q; g < D.ngroups; g += LN)
#pragma unroll
        for (int m = 0; m < kNMom; ++m) R[m] += D.mom_part[((size_t)g * kNMom + m) * nx + sc];

    // quadrature tables in LDS, rows of h and He padded with zeros to the unrolled counts: a contiguous
    // copy of the case's image of them (the plan's layout is a prefix of it); every thread issues up
    // to 8 loads before its first LDS write, so the copy takes one memory round trip (up to 2048
    // doubles: every velocity set up to Qx = 80, Nx = 10)
    const CellLds lay = cell_lds(D.qx, D.qy, D.nxb, D.nyb, D.nyo, uses_aux2(D.cell_lanes));
    const gptr<const double> img = gmem(D.ktab);
    constexpr int kStageBatch = 8;
    for (int base = 0; base < lay.total; base += kStageBatch * kCellThreads) {
        double v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int k = base + u * kCellThreads + (int)threadIdx.x;
            v[u] = k < lay.total ? img[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int k = base + u * kCellThreads + (int)threadIdx.x;
            if (k < lay.total) ktab[k] = v[u];
        }
    }
    __syncthreads();

    if (!wall_blocks_of_their_own(D.qx, D.qy)) {
        // walls done by the edge blocks: the block holding cell 0 the left wall, the one holding
        // cell nx-1 the right wall
        if (cr.cell0 == 0) wall_left<T>(D, fcur, flags);
        if (cr.cell0 + kCellThreads / LN >= nx) wall_right<T>(D, fcur);
    }

    cell_tables<T>(D, R, q, LN, s, on, flags, D.sc, (T*)D.cell, ktab, lay, avg);
}

// ---- small-case kernel ---------------------------------------------------------------------------
// One workgroup holds one small case in LDS -- its three state buffers, the per-cell tables of the
// collision, the quadrature tables of eqs. (gx), (gy) and every per-velocity and per-cell constant --
// and runs n_steps full SSP-RK3 steps in one launch.  Per stage: the update of every (velocity, 4-cell
// strip) for both distributions (WENO-5 faces with the wall and mirror ghosts of the tiled path, the
// FP64 Shakhov collision and the FP64 stage combine), which also forms the leaving wall fluxes of
// eq. (diffuse_nw) from the values it stores; then the wall densities, the moments of the new state
// (FP64 sums over every velocity of a cell, split over the cell's lanes) and the per-cell tables
// (cell_tables, as in the per-cell kernel).  For cases of a few thousand cell-velocity units, whose
// tiled steps (six launches) are bound by launch latency; with one block per case, its latency is
// what remains, so nothing it reads inside the step loop comes from global memory.  The step counter,
// the fields of the final state, the running averages, the wall densities and, at a checked last
// step, the residual, the mean P_xy, the mass and the local-time-step rescaling are kept as the tiled
// path keeps them; the numbers are this path's own (another summation order).
constexpr int kSmallThreads = 256;

// LDS layout of a small case (bytes from the start of the dynamic LDS).  The rows of the state buffers
// (one distribution of one velocity) are small_row(nx) = nx + 1 elements apart: with an odd stride the
// rows of neighbouring velocities start on different banks, so that the update's window reads (lanes
// spread over velocities and strips) and the moment sums (lanes spread over velocities and cells) do
// not pile onto a few banks.
__host__ __device__ constexpr int small_row(int nx) { return nx + 1; }
struct SmallLds {
    size_t buf[3], sc, g, ktab, pm, vel, cel, total;
};
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline int small_lanes(int nx)
{
    int ln = kMaxCellLanes;
    while (ln > 1 && ln * nx > kSmallThreads) ln >>= 1;
    return ln;
}
// per-velocity constants [p_x of the 2 Q_x nodes | p_y of the Q_y nodes | g_w left (nv) | g_w right (nv) |
// (p_x, p_y) of every velocity (2 nv)] and per-cell ones [dt_s | residual weight | J deta | 1/(J deta)], FP64
__host__ __device__ inline SmallLds small_lds(int nx, int nv, int qx, int qy, int ktab_total, size_t es)
{
    SmallLds o;
    size_t off = 0;
    for (int k = 0; k < 3; ++k) {
        o.buf[k] = off;
        off = align16(off + es * 2 * (size_t)nv * small_row(nx));
    }
    o.sc = off;
    off = align16(off + sizeof(double) * kNSc * nx);
    o.g = off;
    off = align16(off + es * (size_t)g_slots(qx, qy) * nx);
    o.ktab = off;
    off = align16(off + sizeof(double) * (size_t)ktab_total);
    o.pm = off;  // per cell: n and P_xy of the last analysed state
    off = align16(off + sizeof(double) * 2 * (size_t)nx);
    o.vel = off;
    off = align16(off + sizeof(double) * (size_t)(2 * qx + qy + 4 * nv));
    o.cel = off;
    off = align16(off + sizeof(double) * 4 * (size_t)nx);
    o.total = off;
    return o;
}

// block-wide sums of N values in a fixed order (a shuffle tree per wave, then the waves in order)
template <int N>
__device__ inline void small_block_sum(double (&x)[N], double (*red)[N])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        x[i] = wave_sum(x[i]);
        if (lane == 0) red[wave][i] = x[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int w = 0; w < kSmallThreads / 64; ++w) s += red[w][i];
        x[i] = s;
    }
    __syncthreads();
}

// LDS pointers of a small case
template <typename T>
struct SmallPtrs {
    T *b0, *b1, *b2;                        // state buffers: f^n, stage 1 and stage 2 outputs
    int rs;                                 // their row stride, small_row(nx)
    double* sc;                             // FP64 per-cell scalars [kNSc][nx]
    T* g;                                   // per-cell table [g_slots][nx]
    double* ktab;                           // quadrature tables of eqs. (gx), (gy)
    double* pm;                             // n and P_xy per cell of the last analysed state
    const double *px, *py, *gwl, *gwr;      // per-velocity constants
    const double* pv;                       // (p_x, p_y) of velocity v at 2v, 2v + 1
    const double *dts, *jres, *jdeta;       // per-cell constants
    __device__ __forceinline__ T* buf(int k) const { return k == 0 ? b0 : k == 1 ? b1 : b2; }
};

// Leaving fluxes through both walls (eq. diffuse_nw) of the state f: p_x F and p_x p_y F of the leaving
// face values, F formed exactly as the per-cell kernel's wall blocks form it; velocity v < half leaves
// through the right wall (p_x > 0), v >= half through the left one.  Every wave forms the whole sums
// (lane l takes v = l, l + 64, ..., then a wave sum), so each holds the same bits without a block
// reduction.  w: left flux, left momentum, right flux, right momentum.  (Inside the step loop the
// update forms these sums from the values it stores.)
template <typename T>
__device__ __forceinline__ void small_walls(const InstDesc& D, const SmallPtrs<T>& S, const T* f, double (&w)[4])
{
    const int nx = D.nx, half = D.qx * D.qy;
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = 0.0;
    for (int v = threadIdx.x & 63; v < 2 * half; v += 64) {
        const bool right = v < half;
        if (!right && D.half) continue;
        const T* r = f + (size_t)v * S.rs;
        const T F = right ? wall_face_right(r[nx - 3], r[nx - 2], r[nx - 1]) : wall_face_left(r[0], r[1], r[2]);
        const double pxv = S.pv[2 * v], pyv = S.pv[2 * v + 1];
        const double a = pxv * (double)F, b = pxv * pyv * (double)F;
        if (right) {
            w[2] += a;
            w[3] += b;
        } else {
            w[0] += a;
            w[1] += b;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = wave_sum(w[i]);
}

// moments and per-cell tables of the state f (block-wide) and the wall densities from its wall sums w
// (identical in every thread); flags as the per-cell kernel's; returns the wall densities and the
// y-momentum fluxes through the walls (stored once per launch)
template <typename T>
__device__ __forceinline__ void small_analyze(const InstDesc& D, const SmallPtrs<T>& S, const T* f, const CellLds& lay, int LN,
                              int flags, const double (&w)[4], double& nwl, double& nwr, double& shl, double& shr, int avg)
{
    const int nx = D.nx, nv = D.nv;
    const int tid = threadIdx.x;
    nwl = D.half ? 0.0 : -w[0] / D.den_l;
    nwr = -w[2] / D.den_r;
    const int q = tid % LN;
#pragma unroll 1
    for (int c0 = 0; c0 < nx; c0 += kSmallThreads / LN) {
        const int s = c0 + tid / LN;
        const bool on = s < nx;
        const int sc_ = on ? s : 0;
        // raw sums of Sec. II's moments over the velocities of the cell, lane q taking the block
        // v = q vb ... q vb + vb - 1 (the rows of a block are consecutive, one bank apart)
        double R[kNMom];
#pragma unroll
        for (int m = 0; m < kNMom; ++m) R[m] = 0.0;
        const int vb = (nv + LN - 1) / LN, vend = min(nv, (q + 1) * vb);
        for (int v = q * vb; v < vend; ++v) {
            const double pxv = S.pv[2 * v], pyv = S.pv[2 * v + 1];
            const double o = (double)f[(size_t)v * S.rs + sc_], x = (double)f[(size_t)(nv + v) * S.rs + sc_];
            const double p2 = pxv * pxv + pyv * pyv;
            R[0] += o;
            R[1] += pxv * o;
            R[2] += pyv * o;
            R[3] += pxv * pxv * o;
            R[4] += pxv * pyv * o;
            R[5] += pyv * pyv * o;
            R[6] += p2 * pxv * o;
            R[7] += p2 * pyv * o;
            R[8] += x;
            R[9] += pxv * x;
            R[10] += pyv * x;
        }
        cell_tables<T, true>(D, R, q, LN, s, on, flags, S.sc, S.g, S.ktab, lay, avg);
        if (on && q == 0) {
            // the same arithmetic as the fields of cell_tables: n and P_xy of the cell
            const double n = R[0], ux = R[1] / n, uy = R[2] / n;
            S.pm[s] = n;
            S.pm[nx + s] = R[4] - n * ux * uy;
        }
    }
    shl = D.half ? 0.0 : w[1] + nwl * D.mom_l;
    shr = w[3] + nwr * D.mom_r;
    __syncthreads();
}

// one SSP-RK3 stage from fin (f^n in S.b0) into fout, each item one velocity over 4 cells, both
// distributions (phi and chi share the velocity's constants, the cells' tables and the collision's
// common terms; their two WENO windows are independent work); residual partials on request.  The
// items that store a wall's three cells of a leaving velocity also form its leaving face value of phi
// (as small_walls does, from the stored values), so that w returns the wall sums of fout, identical in
// every thread (thread partials, wave sums, then the waves in order through red).
template <typename T>
__device__ __forceinline__ void small_update(const InstDesc& D, const SmallPtrs<T>& S, const T* fin, T* fout, int stage,
                             uint32_t stepc, bool want_res, double nwl, double nwr, double& rnum, double& rden,
                             double (*red)[4], double (&w)[4])
{
    const int nx = D.nx, nv = D.nv, qx = D.qx, qy = D.qy, half = qx * qy;
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = 0.0;
    const double ca = stage == 1 ? 0.75 : stage == 2 ? (1.0 / 3.0) : 0.0;
    const double cb = stage == 1 ? 0.25 : stage == 2 ? (2.0 / 3.0) : 1.0;
    const uint32_t rkey = D.rounding ? hash32(D.seed ^ hash32(stepc * 3u + (uint32_t)stage + 0x9e3779b9u)) : 0u;
    const int nstrip = nx / kStrip, per_dist = nv * nstrip;
    const T* fn = S.b0;
#pragma unroll 1
    for (int r = threadIdx.x; r < per_dist; r += kSmallThreads) {
        const int v = r / nstrip, s0 = (r - v * nstrip) * kStrip;
        const int hi = v / qy, j = v - hi * qy;
        const double pxd = S.px[hi], pyd = S.py[j];
        const T pxt = (T)pxd;
        const bool first = s0 == 0 && !D.half, mirror = s0 == 0 && D.half, last = s0 + kStrip == nx;
        size_t row[2];
        Win<T> P[2];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            row[d] = (size_t)(d * nv + v) * S.rs;
            const T* fr = fin + row[d];
            // window cells s0-4 .. s0+7; the tiled path's loads: cells 0..3 for the left window of the
            // strip at cell 0, cells s0..s0+3 for the right window of the last strip (the ghost logic
            // below replaces whatever of them the faces read)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                P[d].w[c] = fr[s0 == 0 ? c : s0 - 4 + c];
                P[d].w[4 + c] = fr[s0 + c];
                P[d].w[8 + c] = fr[last ? s0 + c : s0 + 4 + c];
            }
        }
        if (mirror) {
            // point symmetry of Sec. II about x = 0: ghost cells -1..-4 of (p_x, p_y) hold the values of
            // (-p_x, -p_y) in cells 0..3
            const int hmir = hi < qx ? hi + qx : hi - qx;
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const T* fm = fin + (size_t)(d * nv + hmir * qy + (qy - 1 - j)) * S.rs;
#pragma unroll
                for (int c = 0; c < 4; ++c) P[d].w[3 - c] = fm[c];
            }
        }
        // every table value and f^n of the 4 cells read before the first store: in FP64 the tables
        // and the state share a type, so reads after a store would wait for it
        double ux[kStrip], uy[kStrip], itau[kStrip], A5[kStrip], qxv[kStrip], qyv[kStrip], tt[kStrip];
        double s8[kStrip], s4[kStrip], dts[kStrip], fnd[2][kStrip];
        T ijd[kStrip], gy[kStrip], gx[kStrip];
#pragma unroll
        for (int c = 0; c < kStrip; ++c) {
            const int s = s0 + c;
            const double* sc = S.sc + s;
            ux[c] = sc[SC_UX * nx];
            uy[c] = sc[SC_UY * nx];
            itau[c] = sc[SC_INVTAU * nx];
            A5[c] = sc[SC_AS5T * nx];
            qxv[c] = sc[SC_QX * nx];
            qyv[c] = sc[SC_QY * nx];
            tt[c] = sc[SC_T * nx];
            s8[c] = sc[SC_S8 * nx];
            s4[c] = sc[SC_S4 * nx];
            ijd[c] = S.g[kGIjd * nx + s];
            gy[c] = S.g[(kGx0 + 2 * qx + j) * nx + s];
            gx[c] = S.g[(kGx0 + hi) * nx + s];
            dts[c] = S.dts[s];
#pragma unroll
            for (int d = 0; d < 2; ++d) fnd[d][c] = stage > 0 ? (double)fn[row[d] + s] : 0.0;
        }
        // wall populations (eq. diffuse): n_w g_w for phi, T_w n_w g_w for chi
        T F[2][5];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const double sl = d ? D.Tw * nwl : nwl, sr = d ? D.Tw * nwr : nwr;
            const T wl = first ? (T)(sl * S.gwl[v]) : T(0), wr = last ? (T)(sr * S.gwr[v]) : T(0);
            if (pxt > T(0)) {
                if (first) P[d].w[1] = P[d].w[2] = P[d].w[3] = wl;
                if (last) {
                    P[d].w[8] = ext_p3(P[d].w[5], P[d].w[6], P[d].w[7]);
                    P[d].w[9] = ext_p4(P[d].w[5], P[d].w[6], P[d].w[7]);
                }
                P[d].faces_pos(F[d]);
                if (first) F[d][0] = wl;
            } else {
                if (first) {
                    P[d].w[3] = ext_m1(P[d].w[4], P[d].w[5], P[d].w[6]);
                    P[d].w[2] = ext_m2(P[d].w[4], P[d].w[5], P[d].w[6]);
                }
                if (last) P[d].w[8] = P[d].w[9] = P[d].w[10] = wr;
                P[d].faces_neg(F[d]);
                if (last) F[d][4] = wr;
            }
        }
        uint32_t rbits[kStrip] = {0, 0, 0, 0};
        if (D.rounding) {
            const uint32_t base = rkey ^ ((uint32_t)v * 0x85ebca6bu) ^ ((uint32_t)s0 * 0xc2b2ae35u);
#pragma unroll
            for (int c = 0; c < kStrip; ++c) rbits[c] = c == 0 ? hash32(base) : weyl32(rbits[c - 1]);
        }
        T st[kStrip];  // the stored phi values
#pragma unroll
        for (int c = 0; c < kStrip; ++c) {
            const int s = s0 + c;
            // reduced Shakhov collision, Sec. II, in FP64 (the same operations as the tiled path): phi
            // relaxes to V - 0.8 A W = phi_eq (1 + S_phi), chi to T (V - 0.4 A W) = T phi_eq (1 + S_chi)
            const double xx = pxd - ux[c], xy = pyd - uy[c];
            const double x2 = xx * xx + xy * xy;
            const double qxi = qxv[c] * xx + qyv[c] * xy;
            const double feq = (double)gx[c] * (double)gy[c];
            const double W = feq * qxi;
            const double V = fma(W, A5[c] * x2, feq);
            const double tg[2] = {fma(-W, s8[c], V), tt[c] * fma(-W, s4[c], V)};
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const T fv = P[d].w[4 + c];
                const T a = (F[d][c + 1] - F[d][c]) * (-pxt * ijd[c]);
                const double L = (double)a + (tg[d] - (double)fv) * itau[c];
                const double oe = ca * fnd[d][c] + cb * ((double)fv + dts[c] * L);
                // stage 3 writes f^n in place: f^n is read only at an item's own cells, by that item
                const T o = store_round<T>(oe, D.rounding, d ? rbits[c] >> 16 : rbits[c]);
                if (d == 0) st[c] = o;
                fout[row[d] + s] = o;
                if (want_res) {
                    const double dd = oe - fnd[d][c];
                    rnum += S.jres[s] * (dd * dd);
                    rden += S.jdeta[s] * (fnd[d][c] * fnd[d][c]);
                }
            }
        }
        // cells nx-3..nx-1 are cells 1..3 of the last strip, cells 0..2 those of the first
        if (last && v < half) {
            const T Fw = wall_face_right(st[1], st[2], st[3]);
            w[2] += pxd * (double)Fw;
            w[3] += pxd * pyd * (double)Fw;
        }
        if (first && v >= half) {
            const T Fw = wall_face_left(st[0], st[1], st[2]);
            w[0] += pxd * (double)Fw;
            w[1] += pxd * pyd * (double)Fw;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = wave_sum(w[i]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[threadIdx.x >> 6][i] = w[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double t = 0.0;
        for (int k = 0; k < kSmallThreads / 64; ++k) t += red[k][i];
        w[i] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kSmallThreads) void small_kernel(const InstDesc* __restrict__ descs, int n_steps,
                                                                int check)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ double red[kSmallThreads / 64][4];
    const InstDesc& D = descs[blockIdx.x];
    const int nx = D.nx, nv = D.nv, qx = D.qx, qy = D.qy;
    const int LN = small_lanes(nx);
    const CellLds lay = cell_lds(qx, qy, D.nxb, D.nyb, D.nyo, uses_aux2(LN));
    const SmallLds L = small_lds(nx, nv, qx, qy, lay.total, sizeof(T));
    double* vel = (double*)(lds + L.vel);
    double* cel = (double*)(lds + L.cel);
    SmallPtrs<T> S;
    S.b0 = (T*)(lds + L.buf[0]);
    S.b1 = (T*)(lds + L.buf[1]);
    S.b2 = (T*)(lds + L.buf[2]);
    S.rs = small_row(nx);
    S.sc = (double*)(lds + L.sc);
    S.g = (T*)(lds + L.g);
    S.ktab = (double*)(lds + L.ktab);
    S.pm = (double*)(lds + L.pm);
    S.px = vel;
    S.py = vel + 2 * qx;
    S.gwl = vel + 2 * qx + qy;
    S.gwr = vel + 2 * qx + qy + nv;
    S.pv = vel + 2 * qx + qy + 2 * nv;
    S.dts = cel;
    S.jres = cel + nx;
    S.jdeta = cel + 2 * nx;
    const int tid = threadIdx.x;
    // the state, the quadrature tables and the constants into LDS
    const T* f0 = (const T*)D.f[0];
    const int nst = 2 * nv * nx;  // the state's elements, rows of nx in global memory
    for (int k = tid; k < nst; k += kSmallThreads) S.b0[(k / nx) * S.rs + k % nx] = f0[k];
    for (int k = tid; k < lay.total; k += kSmallThreads) S.ktab[k] = D.ktab[k];
    for (int k = tid; k < 2 * qx; k += kSmallThreads) vel[k] = D.px[k];
    for (int k = tid; k < qy; k += kSmallThreads) vel[2 * qx + k] = D.py[k];
    for (int k = tid; k < nv; k += kSmallThreads) {
        vel[2 * qx + qy + k] = D.gw_l[k];
        vel[2 * qx + qy + nv + k] = D.gw_r[k];
        vel[2 * qx + qy + 2 * nv + 2 * k] = D.px[k / qy];
        vel[2 * qx + qy + 2 * nv + 2 * k + 1] = D.py[k % qy];
    }
    for (int k = tid; k < nx; k += kSmallThreads) {
        cel[k] = D.dts[k];
        cel[nx + k] = D.jres[k];
        cel[2 * nx + k] = D.jdeta[k];
        S.g[kGIjd * nx + k] = (T)D.inv_jdeta[k];
    }
    __syncthreads();
    // the step counter and the averaging switch, read once: nothing else changes them during the launch
    const double step0 = D.dyn[DY_STEP];
    const int avg = D.dyn[DY_AVG_ON] != 0.0;
    uint32_t stepc = (uint32_t)step0;
    double nwl = 0.0, nwr = 0.0, shl = 0.0, shr = 0.0;
    double w[4];
    small_walls<T>(D, S, S.b0, w);
    small_analyze<T>(D, S, S.b0, lay, LN, 0, w, nwl, nwr, shl, shr, avg);
    double rnum = 0.0, rden = 0.0;
#pragma unroll 1
    for (int k = 0; k < 3 * n_steps; ++k) {
        // stage 1: f^n -> b1; stage 2: (b1, f^n) -> b2; stage 3: (b2, f^n) -> f^n in place
        const int stage = k % 3;
        const bool res = check && k + 1 == 3 * n_steps;
        T* fin = S.buf(stage);
        T* fout = S.buf(stage == 2 ? 0 : stage + 1);
        small_update<T>(D, S, fin, fout, stage, stepc, res, nwl, nwr, rnum, rden, red, w);
        if (stage == 2) ++stepc;
        // the fields of the state at the end of every step are needed only with the running averages
        // on; otherwise those of the launch's last step
        const int fl = stage != 2 ? 0 : (avg ? FLAG_STEP_DONE : 0) | (k + 1 == 3 * n_steps ? FLAG_FIELDS : 0);
        small_analyze<T>(D, S, fout, lay, LN, fl, w, nwl, nwr, shl, shr, avg);
    }
    if (check) {
        // residual, J-weighted mean P_xy and mass of the final state, as the tiled path's check
        double r[4] = {rnum, rden, 0.0, 0.0};
        for (int s = tid; s < nx; s += kSmallThreads) {
            r[2] += S.jdeta[s] * S.pm[nx + s];
            r[3] += S.jdeta[s] * S.pm[s];
        }
        small_block_sum<4>(r, red);
        if (tid == 0) {
            D.dyn[DY_RES_NUM] = r[0];
            D.dyn[DY_RES_DEN] = r[1];
            D.dyn[DY_PXY_MEAN] = r[2] / D.jsum;
            D.dyn[DY_MASS] = r[3];
            const double chk = r[0] + r[1] + r[2] + r[3];
            if (!(chk == chk) || chk - chk != 0.0) D.dyn[DY_FLAGS] = 1.0;
        }
        if (D.lts) {
            // local time steps: back to the rest-state mass, then the moments of the rescaled state
            const double scale = D.jsum / r[3];
            for (int k = tid; k < nst; k += kSmallThreads) {
                T& e = S.b0[(k / nx) * S.rs + k % nx];
                e = (T)((double)e * scale);
            }
            __syncthreads();
            small_walls<T>(D, S, S.b0, w);
            small_analyze<T>(D, S, S.b0, lay, LN, FLAG_FIELDS, w, nwl, nwr, shl, shr, avg);
        }
    }
    if (tid == 0) {
        D.dyn[DY_NWL] = nwl;
        D.dyn[DY_NWR] = nwr;
        D.dyn[DY_SHEAR_L] = shl;
        D.dyn[DY_SHEAR_R] = shr;
        D.dyn[DY_STEP] = step0 + (double)n_steps;
        if (avg) D.dyn[DY_AVG_STEPS] += (double)n_steps;
    }
    T* fo = (T*)D.f[0];
    for (int k = tid; k < nst; k += kSmallThreads) fo[k] = S.b0[(k / nx) * S.rs + k % nx];
}

// ---- per-instance reductions at a check point: residual, mean P_xy, mass ----------------------
// local time steps: after a checked step (DY_MASS from finalize_kernel), the populations of instance
// blockIdx.y are rescaled to the rest-state mass sum_s J_s deta; other instances are left alone
template <typename T>
__global__ __launch_bounds__(256) void renorm_kernel(const InstDesc* __restrict__ descs)
{
    const InstDesc& D = descs[blockIdx.y];
    if (!D.lts) return;
    const double scale = D.jsum / D.dyn[DY_MASS];
    T* f = (T*)D.f[0];
    const size_t n = 2 * (size_t)D.nv * (size_t)D.nx;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        f[k] = (T)((double)f[k] * scale);
}

__global__ __launch_bounds__(256) void finalize_kernel(const InstDesc* __restrict__ descs, int with_res)
{
    __shared__ double red[256][4];
    const InstDesc& D = descs[blockIdx.x];
    const int nx = D.nx;
    double a = 0, b = 0, c = 0, d = 0;
    if (with_res) {
        const int nt = D.nctiles * D.ngroups;
        for (int t = threadIdx.x; t < nt; t += 256) {
            a += D.res_part[t * 2 + 0];
            b += D.res_part[t * 2 + 1];
        }
    }
    for (int s = threadIdx.x; s < nx; s += 256) {
        c += D.jdeta[s] * D.fields[F_PXY * nx + s];
        d += D.jdeta[s] * D.fields[F_N * nx + s];
    }
    red[threadIdx.x][0] = a;
    red[threadIdx.x][1] = b;
    red[threadIdx.x][2] = c;
    red[threadIdx.x][3] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[threadIdx.x][q] += red[threadIdx.x + w][q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double jsum = D.jsum;
        if (with_res) {
            D.dyn[DY_RES_NUM] = red[0][0];
            D.dyn[DY_RES_DEN] = red[0][1];
        }
        D.dyn[DY_PXY_MEAN] = red[0][2] / jsum;
        D.dyn[DY_MASS] = red[0][3];
        const double chk = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        if (!(chk == chk) || chk - chk != 0.0) D.dyn[DY_FLAGS] = 1.0;
    }
}

// ---- time averages of the fields: start (clear the sums and the count, switch on) or stop ------
__global__ __launch_bounds__(256) void average_kernel(const InstDesc* __restrict__ descs, int start)
{
    const InstDesc& D = descs[0];
    if (start) {
        const int n = kNFields * D.nx;
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) D.avg[k] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        D.dyn[DY_AVG_ON] = start ? 1.0 : 0.0;
        if (start) D.dyn[DY_AVG_STEPS] = 0.0;
    }
}

// ---- state initialisation: rest equilibrium phi = g0[v], chi = T_w g0[v] -----------------------
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(const InstDesc* __restrict__ descs, int inst)
{
    const InstDesc& D = descs[inst];
    const size_t total = (size_t)D.nv * D.nx;
    T* f0 = (T*)D.f[0];
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const int v = (int)(k / D.nx);
        const double g = D.g0[v];
        f0[k] = (T)g;
        f0[total + k] = (T)(D.Tw * g);
    }
}

}  // namespace hrlb

// ---- static scratch of the allocation-free case (hrlb_init_case_static) ---------------------------
// The auxiliary region of one case (descriptor, tables, cell tables, fields, moment and residual
// partials, work lists, counters) for callers that cannot allocate device memory.  Every device the
// library runs on holds its own copy until the process ends.
namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kScratchDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of the current device's scratch (looked up once per device with that device current;
// the array's name is a host-side stand-in, not a device address) and its size.
extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_scratch(void** ptr, size_t* bytes)
{
    static std::mutex mu;
    static void* addr[kScratchDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

// ---- host-callable launchers (C linkage inside the library) --------------------------------------
using namespace hrlb;

// dynamic LDS of the stage kernel for a batch whose largest full-range order is qy_max
extern "C" __attribute__((visibility("hidden"))) size_t hrlbk_stage_lds(int fp32, int qy_max)
{
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    // FP32: the cell tables are followed by p_y and the wall populations of the tile's velocities
    const size_t vel =
        fp32 ? sizeof(double) * (size_t)qy_max + sizeof(float) * (size_t)(2 * kRows * std::min(qy_max, kMaxVpt)) : 0;
    const size_t cells = cell_lds_bytes(qy_max, es) + vel;
    const size_t moms = sizeof(double) * moments_per_pass(fp32 ? sizeof(float) : sizeof(double)) * kRows * kTileCells;
    return cells > moms ? cells : moms;
}

namespace {
// blocks of one stage-kernel variant that fit on the device at once, as a multiple of the XCD count
template <typename T, int MODE>
int resident_grid(size_t lds)
{
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, lds});
    if (it != cache.end()) return it->second;
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)stage_kernel<T, MODE>, kThreads, lds) !=
            hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    const int g = std::max(kXcds, (std::max(1, per_cu) * ncu) / kXcds * kXcds);
    cache.emplace(std::make_pair(dev, lds), g);
    return g;
}

template <typename T, int MODE>
hipError_t launch_stage(const InstDesc* descs, const TileRef* tiles, int ntiles, int stage, unsigned* ctr, size_t lds,
                        hipStream_t st)
{
    int grid = resident_grid<T, MODE>(lds);
    if (grid < 0) return hipErrorInvalidValue;
    grid = std::min(grid, std::max(kXcds, (ntiles + kXcds - 1) / kXcds * kXcds));  // a tile list is 8k long
    hipLaunchKernelGGL((stage_kernel<T, MODE>), dim3(grid), dim3(kThreads), lds, st, descs, tiles, ntiles, stage, ctr);
    return hipGetLastError();
}
}  // namespace

// ctr: kXcds + 1 zeroed counters owned by the caller's launch list (the kernel leaves them zeroed)
extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_stage(int fp32, const InstDesc* descs, const TileRef* tiles, int ntiles,
                                  unsigned* ctr, int stage, int flags, int qy_max, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const size_t lds = hrlbk_stage_lds(fp32, qy_max);
    if (stage < 0)
        return fp32 ? launch_stage<float, kModeAnalyze>(descs, tiles, ntiles, 0, ctr, lds, st)
                    : launch_stage<double, kModeAnalyze>(descs, tiles, ntiles, 0, ctr, lds, st);
    if ((flags & FLAG_RESID) && stage == 2)
        return fp32 ? launch_stage<float, kModeResid>(descs, tiles, ntiles, stage, ctr, lds, st)
                    : launch_stage<double, kModeResid>(descs, tiles, ntiles, stage, ctr, lds, st);
    if (stage == 0)
        return fp32 ? launch_stage<float, kModeStep0>(descs, tiles, ntiles, stage, ctr, lds, st)
                    : launch_stage<double, kModeStep0>(descs, tiles, ntiles, stage, ctr, lds, st);
    return fp32 ? launch_stage<float, kModeStep>(descs, tiles, ntiles, stage, ctr, lds, st)
                : launch_stage<double, kModeStep>(descs, tiles, ntiles, stage, ctr, lds, st);
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_cell(int fp32, const InstDesc* descs, const CellRef* cells, int ncells, int buf,
                                 int flags, size_t shmem, hipStream_t st)
{
    if (ncells <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(cell_kernel<float>, dim3(ncells), dim3(kCellThreads), shmem, st, descs, cells, buf, flags);
    else
        hipLaunchKernelGGL(cell_kernel<double>, dim3(ncells), dim3(kCellThreads), shmem, st, descs, cells, buf, flags);
    return hipGetLastError();
}

// bytes of dynamic LDS the small-case kernel needs for one instance
extern "C" __attribute__((visibility("hidden"))) size_t hrlbk_small_lds(const InstDesc* D)
{
    const int LN = small_lanes(D->nx);
    const CellLds lay = cell_lds(D->qx, D->qy, D->nxb, D->nyb, D->nyo, uses_aux2(LN));
    return small_lds(D->nx, D->nv, D->qx, D->qy, lay.total, D->precision == 1 ? sizeof(float) : sizeof(double)).total;
}

// n_steps steps of every small instance of descs (one block each); check: the last step is checked
// dynamic LDS a small-case block may take on the current device: the device's LDS per workgroup less
// the kernel's static LDS (160 KB less a few hundred bytes on MI355X); both kernel variants are
// allowed that much once per device.  0 if the device cannot be queried.
extern "C" __attribute__((visibility("hidden"))) size_t hrlbk_small_lds_max()
{
    static std::mutex mu;
    static std::map<int, size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int per_block = 0;
    hipFuncAttributes fa32{}, fa64{};
    if (hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&fa32, (const void*)small_kernel<float>) != hipSuccess ||
        hipFuncGetAttributes(&fa64, (const void*)small_kernel<double>) != hipSuccess)
        return 0;
    const size_t stat = std::max(fa32.sharedSizeBytes, fa64.sharedSizeBytes);
    size_t lim = per_block > 0 && (size_t)per_block > stat ? (size_t)per_block - stat : 0;
    if (hipFuncSetAttribute((const void*)small_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)small_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) !=
            hipSuccess)
        lim = std::min(lim, size_t(64) << 10);  // keep to the default limit if the opt-in is refused
    cache.emplace(dev, lim);
    return lim;
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_small(int fp32, const InstDesc* descs, int ninst,
                                                                          int n_steps, int check, size_t lds,
                                                                          hipStream_t st)
{
    if (ninst <= 0 || n_steps <= 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(small_kernel<float>, dim3(ninst), dim3(kSmallThreads), lds, st, descs, n_steps, check);
    else
        hipLaunchKernelGGL(small_kernel<double>, dim3(ninst), dim3(kSmallThreads), lds, st, descs, n_steps, check);
    return hipGetLastError();
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_renorm(int fp32, const InstDesc* descs, int ninst, hipStream_t st)
{
    for (int i0 = 0; i0 < ninst; i0 += 65535) {  // gridDim.y is at most 65535
        const dim3 grid(256, (unsigned)std::min(65535, ninst - i0));
        if (fp32)
            hipLaunchKernelGGL(renorm_kernel<float>, grid, dim3(256), 0, st, descs + i0);
        else
            hipLaunchKernelGGL(renorm_kernel<double>, grid, dim3(256), 0, st, descs + i0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_finalize(const InstDesc* descs, int ninst, int with_res, hipStream_t st)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(ninst), dim3(256), 0, st, descs, with_res);
    return hipGetLastError();
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_average(const InstDesc* desc, int start, int nx,
                                                                            hipStream_t st)
{
    const int grid = start ? (kNFields * nx + 255) / 256 : 1;
    hipLaunchKernelGGL(average_kernel, dim3(grid), dim3(256), 0, st, desc, start);
    return hipGetLastError();
}

extern "C" __attribute__((visibility("hidden"))) hipError_t hrlbk_init(int fp32, const InstDesc* descs, int inst, size_t units, hipStream_t st)
{
    int grid = (int)((units + 255) / 256);
    if (grid > 65535) grid = 65535;
    if (grid < 1) grid = 1;
    if (fp32)
        hipLaunchKernelGGL(init_kernel<float>, dim3(grid), dim3(256), 0, st, descs, inst);
    else
        hipLaunchKernelGGL(init_kernel<double>, dim3(grid), dim3(256), 0, st, descs, inst);
    return hipGetLastError();
}
