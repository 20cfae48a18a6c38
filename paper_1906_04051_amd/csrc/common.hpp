// Internal device/host definitions shared by the HIP translation units of the
// deflated GMRES(m) library.  Not part of the public interface (include/gmres.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gm {

constexpr int kWG = 256;            // threads per workgroup of the streaming kernels
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kMaxM = 96;           // largest supported restart length m
constexpr int kMaxR = 256;          // largest deflation count per system (coarse solve in one WG)
constexpr int kAzRowMax = 64;       // largest row length of the compact A*Z operator
constexpr int kBlockColsMax = 64;   // deflation columns per SpMV row block (fused Z^T y)
constexpr int kXcd = 8;             // accelerator complex dies (own L2 each); blocks go round-robin

// ------------------------------------------------------ bounds-checking build
// Built with -DGMRES_DEBUG (`python -m paper_1906_04051_amd.build --debug`),
// GM_DCHECK(cond, bit) ORs `bit` into this translation unit's device flag word
// when cond fails and lets the kernel go on; after every API call the host
// waits for the plan's stream, reads and clears the words of every unit and
// returns GMRES_EDEVICE naming the bits.  Release builds compile the checks
// away.  Bits: column index of a CSR row, of a sliced-ELL row, deflation
// column of a Z or A Z entry, slot range of the fused Z^T y partials, column
// of a batched system's row outside its system, column of the block SpMM.
constexpr unsigned kDbgCsrCol = 1u, kDbgSellCol = 2u, kDbgDeflCol = 4u, kDbgSlot = 8u,
                   kDbgBatchCol = 16u, kDbgBlockCol = 32u;
#ifdef GMRES_DEBUG
static __device__ unsigned int g_dbg_flags;
#define GM_DCHECK(cond, bit)                                   \
    do {                                                       \
        if (!(cond)) atomicOr(&::gm::g_dbg_flags, (bit));      \
    } while (0)
#define GM_DEBUG_ACCESSOR(fn)                                                              \
    unsigned int fn() {                                                                    \
        unsigned int v = 0, z = 0;                                                         \
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(::gm::g_dbg_flags), sizeof v) != hipSuccess) \
            return 0x80000000u;                                                            \
        if (v && hipMemcpyToSymbol(HIP_SYMBOL(::gm::g_dbg_flags), &z, sizeof z) != hipSuccess) \
            return v | 0x80000000u;                                                        \
        return v;                                                                          \
    }
#else
#define GM_DCHECK(cond, bit) \
    do {                     \
    } while (0)
#define GM_DEBUG_ACCESSOR(fn) \
    unsigned int fn() { return 0; }
#endif

// Device-resident control block of one solve.  Every kernel of a restart
// cycle reads it, so the host launches whole cycles without synchronising.
struct Ctrl {
    int64_t its;          // inner Arnoldi steps so far (all cycles)
    int64_t max_iters;
    int32_t cycles;
    int32_t stop;         // current cycle has ended (converged estimate, breakdown or cap)
    int32_t done;         // solve has ended
    int32_t status;       // gmres_status at exit
    int32_t k;            // number of basis vectors used by the current cycle
    int32_t breakdown;
    double rho0;          // ||b - A x0||
    double target;        // rtol * rho0
    double beta;          // ||P r|| at the last restart
    double wpre2;         // ||P A v_j||^2 before orthogonalisation (breakdown test)
    double inner_scale;   // mixed precision: ||r|| of the current refinement
    int32_t est_conv;     // some cycle's estimate |gamma_{k+1}| met the target
    int32_t pad32;
    int64_t hist_base;    // history index of this run's first step (earlier runs of the same solve)
    int64_t pad[2];
};

// A kernel returns at once when the solve (gate 1) or the current cycle
// (gate 2) has ended; gate 0 always runs.
__device__ __forceinline__ bool gated(const Ctrl* c, int gate) {
    if (gate == 0 || c == nullptr) return false;
    return c->done != 0 || (gate == 2 && c->stop != 0);
}

// ---------------------------------------------------------------- reductions

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over a workgroup of kWG threads; result valid in every thread.
// `lds` needs kWG / kWave entries.  Fixed order: butterfly within waves,
// then waves 0..3 in order.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    T s = lds[0];
#pragma unroll
    for (int i = 1; i < kWG / kWave; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// Sum over a workgroup of NT threads (fixed order), valid in every thread.
template <int NT, typename T>
__device__ __forceinline__ T block_sum_n(T v, T* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    T s = lds[0];
#pragma unroll
    for (int i = 1; i < NT / kWave; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// Workgroup b of nb runs on die b % kXcd.  Returns a bijection of [0, nb)
// under which each die's workgroups, in dispatch order, take one contiguous
// range of logical blocks, so neighbouring rows (and the vector entries
// they gather) meet in the same die's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % kXcd, k = b / kXcd;
    const int q = nb / kXcd, r = nb % kXcd;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Half-precision basis storage helpers.
__device__ __forceinline__ float ld_f(const __half* p) { return __half2float(*p); }
__device__ __forceinline__ float ld_f(const float* p) { return *p; }
__device__ __forceinline__ double ld_f(const double* p) { return *p; }
__device__ __forceinline__ void st_v(__half* p, float v) { *p = __float2half_rn(v); }
__device__ __forceinline__ void st_v(float* p, float v) { *p = v; }
__device__ __forceinline__ void st_v(double* p, double v) { *p = v; }

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace gm
