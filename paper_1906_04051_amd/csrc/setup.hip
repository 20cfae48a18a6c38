// Setup kernels of a solver plan: input validation, CSR transposes (Z^T and,
// for the adjoint, A^T), the compact coarse operator A Z, the coarse matrix
// E = Z^T A Z per system and its explicit inverse through an LU factorisation
// with partial pivoting (the coarse matrix is the analogue of the paper's
// T_r = U^T A U, arXiv 1906.04051 Sec. 3.3, eq. tau_mat).
//
// All pattern work is deterministic: transposes use a stable radix sort (its
// own kernels below), A Z rows accumulate in CSR order, E entries in Z^T
// order.
#include <vector>

#include "internal.hpp"

namespace gm {

__device__ __forceinline__ int sys_of_row(const int64_t* off, int nsys, int64_t i) {
    int lo = 0, hi = nsys;           // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// flags bit 0: malformed CSR, index out of the row's system block, column
// indices of a row not strictly increasing (unsorted or duplicate);
// bit 1: non-finite value.
__global__ void k_validate(int nsys, int64_t n, int64_t nnz, int64_t znnz,
                           const int64_t* __restrict__ row_off, const int64_t* __restrict__ zcol_off,
                           const int* __restrict__ rowptr, const int* __restrict__ colind,
                           const double* __restrict__ vals, const int* __restrict__ zrp,
                           const int* __restrict__ zci, const double* __restrict__ zv,
                           int* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (rowptr[0] != 0 || (int64_t)rowptr[n] != nnz) atomicOr(flags, 1);
        if (zrp && (zrp[0] != 0 || (int64_t)zrp[n] != znnz)) atomicOr(flags, 1);
    }
    if (i >= n) return;
    const int s = sys_of_row(row_off, nsys, i);
    const int64_t c0 = row_off[s], c1 = row_off[s + 1];
    int f = 0;
    const int k0 = rowptr[i], k1 = rowptr[i + 1];
    if (k1 < k0 || k0 < 0 || (int64_t)k1 > nnz) {
        f |= 1;
    } else {
        int prev = -1;
        for (int k = k0; k < k1; ++k) {
            const int c = colind[k];
            if (c < c0 || c >= c1 || c <= prev) f |= 1;   // in the block, sorted, no duplicates
            prev = c;
            if (!isfinite(vals[k])) f |= 2;
        }
    }
    if (zrp) {
        const int q0 = zrp[i], q1 = zrp[i + 1];
        const int64_t a0 = zcol_off[s], a1 = zcol_off[s + 1];
        if (q1 < q0 || q0 < 0 || (int64_t)q1 > znnz) {
            f |= 1;
        } else {
            int prev = -1;
            for (int q = q0; q < q1; ++q) {
                const int a = zci[q];
                if (a < a0 || a >= a1 || a <= prev) f |= 1;
                prev = a;
                if (!isfinite(zv[q])) f |= 2;
            }
        }
    }
    if (f) atomicOr(flags, f);
}

int setup_validate(const SetupArgs& a, int* d_flags) {
    if (hipMemsetAsync(d_flags, 0, sizeof(int), a.st) != hipSuccess) return kStatusDevice;
    const int64_t nb = (a.n + kWG - 1) / kWG;
    k_validate<<<(unsigned)std::max<int64_t>(nb, 1), kWG, 0, a.st>>>(
        a.nsys, a.n, a.nnz, a.znnz, a.d_sys_row_off, a.d_sys_zcol_off, a.rowptr, a.colind, a.vals,
        a.R > 0 ? a.zrp : nullptr, a.zci, a.zv, d_flags);
    int h = 0;
    if (hipMemcpyAsync(&h, d_flags, sizeof(int), hipMemcpyDeviceToHost, a.st) != hipSuccess ||
        hipStreamSynchronize(a.st) != hipSuccess)
        return kStatusDevice;
    if (h & 1) return kStatusInval;
    if (h & 2) return kStatusNonFinite;
    return kStatusOk;
}

// ------------------------------------------------------------- transpose

__global__ void k_row_of(int64_t n, const int* __restrict__ rowptr, int* __restrict__ row_of) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) row_of[k] = (int)i;
}

// trowptr[c] = first position q with key[q] >= c (keys sorted).
__global__ void k_bounds(int64_t nnz, int64_t ncols, const int* __restrict__ keys,
                         int* __restrict__ trowptr) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > nnz) return;
    const int64_t prev = (q == 0) ? -1 : keys[q - 1];
    const int64_t cur = (q == nnz) ? ncols : keys[q];
    for (int64_t c = prev + 1; c <= cur; ++c) trowptr[c] = (int)q;
}

__global__ void k_take_rows(int64_t nnz, const int* __restrict__ perm, const int* __restrict__ row_of,
                            int* __restrict__ tcolind) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) tcolind[q] = row_of[perm[q]];
}

__global__ void k_gather(int64_t nnz, const int* __restrict__ perm, const double* __restrict__ src,
                         double* __restrict__ dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) dst[q] = src[perm[q]];
}

static unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>((n + kWG - 1) / kWG, 1); }

// ------------------------------------------------------------------ scan
// Exclusive scan of int32 counts in three launches: per-workgroup scans of
// kScanTile entries (with the tile totals in int64), one workgroup scanning
// the tile totals in order, then the tile offsets added.  Integer sums, so the
// result does not depend on the order.

constexpr int kScanTile = 1024;   // entries per workgroup (4 per thread)

__global__ __launch_bounds__(kWG) void k_scan_tiles(int64_t count, const int* __restrict__ in,
                                                    int* __restrict__ out, int64_t* __restrict__ tot) {
    __shared__ int64_t lds[kWG];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
    int v[4];
    int64_t s = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        v[u] = t0 + u < count ? in[t0 + u] : 0;
        s += v[u];
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread sums.
    for (int o = 1; o < kWG; o <<= 1) {
        const int64_t add = threadIdx.x >= o ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = lds[threadIdx.x] - s;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (t0 + u < count) out[t0 + u] = (int)run;
        run += v[u];
    }
    if (threadIdx.x == kWG - 1) tot[blockIdx.x] = lds[kWG - 1];
}

// tot[0 .. nt) -> exclusive offsets in place; tot[nt] = grand total.
__global__ __launch_bounds__(kWG) void k_scan_totals(int64_t nt, int64_t* __restrict__ tot) {
    __shared__ int64_t lds[kWG];
    int64_t carry = 0;
    for (int64_t b = 0; b < nt; b += kWG) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < nt ? tot[i] : 0;
        lds[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kWG; o <<= 1) {
            const int64_t add = threadIdx.x >= o ? lds[threadIdx.x - o] : 0;
            __syncthreads();
            lds[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nt) tot[i] = carry + lds[threadIdx.x] - v;
        carry += lds[kWG - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[nt] = carry;
}

__global__ void k_scan_add(int64_t count, const int64_t* __restrict__ tot, int* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (int)((int64_t)out[i] + tot[i / kScanTile]);
}

static int64_t scan_tiles(int64_t count) { return std::max<int64_t>((count + kScanTile - 1) / kScanTile, 1); }

int scan_i32(hipStream_t st, Arena& ar, const int* in, int* out, int64_t count, int64_t* total) {
    const size_t mk = ar.mark();
    const int64_t nt = scan_tiles(count);
    int64_t* tot = ar.temp_n<int64_t>(nt + 1);
    if (!tot) return kStatusNoMem;
    k_scan_tiles<<<(unsigned)nt, kWG, 0, st>>>(count, in, out, tot);
    k_scan_totals<<<1, kWG, 0, st>>>(nt, tot);
    k_scan_add<<<blocks_for(count), kWG, 0, st>>>(count, tot, out);
    int64_t h = 0;
    hipMemcpyAsync(&h, tot + nt, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    const bool ok = hipStreamSynchronize(st) == hipSuccess;
    ar.release(mk);
    if (!ok) return kStatusDevice;
    *total = h;
    return kStatusOk;
}

static size_t scan_temp_bytes(int64_t count) { return Arena::round((scan_tiles(count) + 1) * sizeof(int64_t)); }

// ------------------------------------------------------------- transpose

static int end_bit_for(int64_t ncols) {
    int end_bit = 1;
    while ((int64_t(1) << end_bit) < ncols) ++end_bit;
    return end_bit;
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort of (key, input position) pairs, 8 bits of the key
// per pass.  Each pass: a digit histogram per tile of kRadixTile consecutive
// items; an exclusive scan of the histogram table in digit-major order, so
// digit d of tile t starts after every smaller digit and after digit d of
// the tiles before t; then a scatter in which each item takes its tile's
// next position for its digit plus its rank among the tile's earlier items
// of that digit.  A tile is read in rounds of kWG items; within a round the
// rank is the count of lower lanes of the wavefront with the same digit
// (eight ballots, one per digit bit), plus the counts of the lower
// wavefronts, kept in LDS; the next positions advance by each round's
// totals.  Equal keys therefore keep their input order, and the output does
// not depend on scheduling.
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixRounds = 8;
constexpr int kRadixTile = kWG * kRadixRounds;
static_assert(kRadixBins == kWG, "one thread per digit");

__global__ __launch_bounds__(kWG) void k_radix_hist(int64_t N, const int* __restrict__ keys, int shift,
                                                    int64_t ntiles, int* __restrict__ hist) {
    __shared__ int cnt[kRadixBins];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x;
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = t * kRadixTile + r * kWG + threadIdx.x;
        if (i < N) atomicAdd(&cnt[(keys[i] >> shift) & (kRadixBins - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + t] = cnt[threadIdx.x];
}

// vals_in == nullptr: the values are the input positions (first pass).
__global__ __launch_bounds__(kWG) void k_radix_scatter(int64_t N, const int* __restrict__ keys_in,
                                                       const int* __restrict__ vals_in, int shift,
                                                       int64_t ntiles, const int* __restrict__ offs,
                                                       int* __restrict__ keys_out,
                                                       int* __restrict__ vals_out) {
    constexpr int NW = kWG / kWave;
    __shared__ int next[kRadixBins];          // next output position of each digit in this tile
    __shared__ int wcnt[NW][kRadixBins];      // this round's count per wavefront and digit
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
    const int64_t t = blockIdx.x;
    next[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + t];
    const unsigned long long below = (1ull << ln) - 1ull;
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = t * kRadixTile + r * kWG + threadIdx.x;
        const bool ok = i < N;
        const int key = ok ? keys_in[i] : 0;
        const int val = ok ? (vals_in ? vals_in[i] : (int)i) : 0;
        const int d = (key >> shift) & (kRadixBins - 1);
        unsigned long long m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        for (int q = threadIdx.x; q < NW * kRadixBins; q += kWG) (&wcnt[0][0])[q] = 0;
        __syncthreads();
        const int rank = __popcll(m & below);
        if (ok && rank == 0) wcnt[wv][d] = __popcll(m);
        __syncthreads();
        int pos = 0;
        if (ok) {
            pos = next[d] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
        }
        __syncthreads();   // every lane has read next[] for this round
        {
            int tot = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) tot += wcnt[w][threadIdx.x];
            next[threadIdx.x] += tot;
        }
        if (ok) {
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();   // before the next round clears wcnt
    }
}

static int radix_passes(int end_bit) { return std::max(1, (end_bit + kRadixBits - 1) / kRadixBits); }
static int64_t radix_tiles(int64_t N) { return std::max<int64_t>((N + kRadixTile - 1) / kRadixTile, 1); }

static size_t radix_temp_bytes(int64_t N, int end_bit) {
    const int64_t table = kRadixBins * radix_tiles(N);
    const size_t pong =
        radix_passes(end_bit) > 1 ? 2 * Arena::round(std::max<int64_t>(N, 1) * sizeof(int)) : 0;
    return 2 * Arena::round(table * sizeof(int)) + pong + scan_temp_bytes(table);
}

// keys_out / perm_out (N entries each): the keys sorted stably and the input
// position of each.  Keys must lie in [0, 2^end_bit).
static int radix_sort_pairs(hipStream_t st, Arena& ar, int64_t N, const int* keys_in, int end_bit,
                            int* keys_out, int* perm_out) {
    if (N == 0) return kStatusOk;
    const size_t mk = ar.mark();
    const int P = radix_passes(end_bit);
    const int64_t ntiles = radix_tiles(N);
    const int64_t table = kRadixBins * ntiles;
    int* hist = ar.temp_n<int>(table);
    int* offs = ar.temp_n<int>(table);
    int* kt = P > 1 ? ar.temp_n<int>(N) : nullptr;
    int* vt = P > 1 ? ar.temp_n<int>(N) : nullptr;
    int status = (!hist || !offs || (P > 1 && (!kt || !vt))) ? kStatusNoMem : kStatusOk;
    const int* kin = keys_in;
    const int* vin = nullptr;
    for (int p = 0; p < P && status == kStatusOk; ++p) {
        // The last pass writes the caller's buffers; earlier ones alternate.
        const bool to_out = ((P - 1 - p) % 2) == 0;
        int* ko = to_out ? keys_out : kt;
        int* vo = to_out ? perm_out : vt;
        const int shift = p * kRadixBits;
        k_radix_hist<<<(unsigned)ntiles, kWG, 0, st>>>(N, kin, shift, ntiles, hist);
        int64_t total = 0;
        status = scan_i32(st, ar, hist, offs, table, &total);
        if (status == kStatusOk && total != N) status = kStatusDevice;
        if (status != kStatusOk) break;
        k_radix_scatter<<<(unsigned)ntiles, kWG, 0, st>>>(N, kin, vin, shift, ntiles, offs, ko, vo);
        kin = ko;
        vin = vo;
    }
    if (status == kStatusOk && hipGetLastError() != hipSuccess) status = kStatusDevice;
    ar.release(mk);
    return status;
}

size_t transpose_temp_bytes(int64_t ncols, int64_t nnz) {
    return 2 * Arena::round(std::max<int64_t>(nnz, 1) * sizeof(int)) + radix_temp_bytes(nnz, end_bit_for(ncols));
}

// Transpose of an nrows x ncols CSR pattern: a stable sort of the entries by
// column keeps every row of the transpose in increasing original-row order.
// tperm[q] is the original entry index of transposed entry q.
int build_transpose(hipStream_t st, Arena& ar, int64_t nrows, int64_t ncols, int64_t nnz,
                    const int* rowptr, const int* colind, int* trowptr, int* tcolind, int* tperm) {
    if (nnz == 0) {
        k_bounds<<<1, kWG, 0, st>>>(0, ncols, colind, trowptr);
        return hipGetLastError() == hipSuccess ? kStatusOk : kStatusDevice;
    }
    const size_t mk = ar.mark();
    int* row_of = ar.temp_n<int>(nnz);
    int* keys_out = ar.temp_n<int>(nnz);
    int status = kStatusOk;
    if (!row_of || !keys_out) {
        status = kStatusNoMem;
    } else {
        k_row_of<<<blocks_for(nrows), kWG, 0, st>>>(nrows, rowptr, row_of);
        status = radix_sort_pairs(st, ar, nnz, colind, end_bit_for(ncols), keys_out, tperm);
        if (status == kStatusOk) {
            k_bounds<<<blocks_for(nnz + 1), kWG, 0, st>>>(nnz, ncols, keys_out, trowptr);
            k_take_rows<<<blocks_for(nnz), kWG, 0, st>>>(nnz, tperm, row_of, tcolind);
            if (hipStreamSynchronize(st) != hipSuccess) status = kStatusDevice;
        }
    }
    ar.release(mk);
    return status;
}

void gather_values(hipStream_t st, int64_t nnz, const int* perm, const double* src, double* dst) {
    if (nnz > 0) k_gather<<<blocks_for(nnz), kWG, 0, st>>>(nnz, perm, src, dst);
}

// ------------------------------------------------------------ compact A Z
// Row i of A Z has an entry for every deflation column reached through the
// columns of row i of A; values accumulate in CSR order (A row, then Z row).

__global__ void k_az_count(int64_t n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                           const int* __restrict__ zrp, const int* __restrict__ zci,
                           int* __restrict__ cnt, int* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cols[kAzRowMax];
    int nc = 0;
    bool over = false;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = colind[k];
        for (int q = zrp[j]; q < zrp[j + 1]; ++q) {
            const int a = zci[q];
            bool found = false;
            for (int t = 0; t < nc; ++t) found |= (cols[t] == a);
            if (!found) {
                if (nc < kAzRowMax) cols[nc++] = a;
                else over = true;
            }
        }
    }
    cnt[i] = nc;
    if (over) atomicOr(flags, 1);
}

__global__ void k_az_fill(int64_t n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                          const double* __restrict__ vals, const int* __restrict__ zrp,
                          const int* __restrict__ zci, const double* __restrict__ zv,
                          const int* __restrict__ azrp, int* __restrict__ azci,
                          double* __restrict__ azv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cols[kAzRowMax];
    double acc[kAzRowMax];
    int nc = 0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = colind[k];
        const double aij = vals[k];
        for (int q = zrp[j]; q < zrp[j + 1]; ++q) {
            const int a = zci[q];
            int t = 0;
            while (t < nc && cols[t] != a) ++t;
            if (t == nc) {
                cols[nc] = a;
                acc[nc] = 0.0;
                ++nc;
            }
            acc[t] += aij * zv[q];
        }
    }
    // Sorted by deflation column (insertion sort; rows are short).
    for (int t = 1; t < nc; ++t) {
        const int c = cols[t];
        const double v = acc[t];
        int u = t - 1;
        while (u >= 0 && cols[u] > c) {
            cols[u + 1] = cols[u];
            acc[u + 1] = acc[u];
            --u;
        }
        cols[u + 1] = c;
        acc[u + 1] = v;
    }
    const int o = azrp[i];
    for (int t = 0; t < nc; ++t) {
        azci[o + t] = cols[t];
        azv[o + t] = acc[t];
    }
}

int az_count(const SetupArgs& a, Arena& ar, const int* rowptr, const int* colind, int* az_rowptr,
             int64_t* az_nnz, int* d_flags) {
    const size_t mk = ar.mark();
    int* cnt = ar.temp_n<int>(a.n + 1);
    if (!cnt) return kStatusNoMem;
    hipMemsetAsync(d_flags, 0, sizeof(int), a.st);
    k_az_count<<<blocks_for(a.n), kWG, 0, a.st>>>(a.n, rowptr, colind, a.zrp, a.zci, cnt, d_flags);
    int64_t total = 0;
    int status = scan_i32(a.st, ar, cnt, az_rowptr, a.n, &total);
    if (status == kStatusOk) {
        int fl = 0;
        const int tot32 = (int)std::min<int64_t>(total, INT32_MAX);
        hipMemcpyAsync(&fl, d_flags, sizeof(int), hipMemcpyDeviceToHost, a.st);
        hipMemcpyAsync(az_rowptr + a.n, &tot32, sizeof(int), hipMemcpyHostToDevice, a.st);
        if (hipStreamSynchronize(a.st) != hipSuccess) status = kStatusDevice;
        else if (fl || total >= INT32_MAX) status = kStatusInval;
        *az_nnz = total;
    }
    ar.release(mk);
    return status;
}

size_t az_count_temp_bytes(int64_t n) { return Arena::round((n + 1) * sizeof(int)) + scan_temp_bytes(n); }

void az_fill(const SetupArgs& a, const int* rowptr, const int* colind, const double* vals,
             const int* az_rowptr, int* az_colind, double* az_vals) {
    k_az_fill<<<blocks_for(a.n), kWG, 0, a.st>>>(a.n, rowptr, colind, vals, a.zrp, a.zci, a.zv,
                                                 az_rowptr, az_colind, az_vals);
}

// ------------------------------------------------------- coarse matrix E
// One thread per entry E_s[a][k] = sum_{i in Z^T row a} z_ia (A Z)_{i,k}
// (row-major per system, offsets e_off).
__global__ void k_build_e(int nsys, const int64_t* __restrict__ zcol_off,
                          const int64_t* __restrict__ e_off, const int* __restrict__ ztrp,
                          const int* __restrict__ ztci, const double* __restrict__ ztv,
                          const int* __restrict__ azrp, const int* __restrict__ azci,
                          const double* __restrict__ azv, double* __restrict__ E) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= e_off[nsys]) return;
    const int s = sys_of_row(e_off, nsys, p);
    const int64_t c0 = zcol_off[s];
    const int r = (int)(zcol_off[s + 1] - c0);
    const int64_t loc = p - e_off[s];
    const int a = (int)(loc / r), k = (int)(loc % r);
    const int col = (int)(c0 + k);
    double acc = 0.0;
    for (int q = ztrp[c0 + a]; q < ztrp[c0 + a + 1]; ++q) {
        const int i = ztci[q];
        for (int t = azrp[i]; t < azrp[i + 1]; ++t)
            if (azci[t] == col) acc += ztv[q] * azv[t];
    }
    E[p] = acc;
}

void build_coarse(const SetupArgs& a, const int* ztrp, const int* ztci, const double* ztv,
                  const int* azrp, const int* azci, const double* azv, const int64_t* d_e_off,
                  double* E) {
    int64_t total = 0;
    hipMemcpyAsync(&total, d_e_off + a.nsys, sizeof(int64_t), hipMemcpyDeviceToHost, a.st);
    hipStreamSynchronize(a.st);
    if (total > 0)
        k_build_e<<<blocks_for(total), kWG, 0, a.st>>>(a.nsys, a.d_sys_zcol_off, d_e_off, ztrp, ztci,
                                                      ztv, azrp, azci, azv, E);
}

// LU with partial pivoting of each E_s (row-major, in place; one workgroup per
// system), then the explicit inverse column by column, stored column-major
// (Einv_s[a*r + i] = (E_s^{-1})_{i,a}).  Pivot = first row of largest |.|;
// singular when |pivot| <= r * eps * max|E_s| (flags bit 2).
__global__ __launch_bounds__(kWG) void k_lu_inverse(const int64_t* __restrict__ zcol_off,
                                                    const int64_t* __restrict__ e_off,
                                                    double* __restrict__ Eall,
                                                    double* __restrict__ Einv_all,
                                                    int* __restrict__ flags) {
    const int s = blockIdx.x;
    const int r = (int)(zcol_off[s + 1] - zcol_off[s]);
    if (r == 0) return;
    double* E = Eall + e_off[s];
    double* X = Einv_all + e_off[s];
    __shared__ double rv[kWG];
    __shared__ int ri[kWG];
    __shared__ int piv[kMaxR];
    __shared__ int sing;
    // max |E|
    double mx = 0.0;
    for (int64_t q = threadIdx.x; q < (int64_t)r * r; q += kWG) mx = fmax(mx, fabs(E[q]));
    rv[threadIdx.x] = mx;
    __syncthreads();
    for (int o = kWG / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) rv[threadIdx.x] = fmax(rv[threadIdx.x], rv[threadIdx.x + o]);
        __syncthreads();
    }
    const double tiny = (double)r * 2.220446049250313e-16 * rv[0];
    if (threadIdx.x == 0) sing = 0;
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        double best = -1.0;
        int bi = r;
        for (int i = k + threadIdx.x; i < r; i += kWG) {
            const double v = fabs(E[(int64_t)i * r + k]);
            if (v > best) { best = v; bi = i; }
        }
        rv[threadIdx.x] = best;
        ri[threadIdx.x] = bi;
        __syncthreads();
        for (int o = kWG / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                const double b2 = rv[threadIdx.x + o];
                const int i2 = ri[threadIdx.x + o];
                if (b2 > rv[threadIdx.x] || (b2 == rv[threadIdx.x] && i2 < ri[threadIdx.x])) {
                    rv[threadIdx.x] = b2;
                    ri[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        const int p = ri[0];
        if (threadIdx.x == 0) {
            piv[k] = p;
            if (!(rv[0] > tiny)) sing = 1;
        }
        __syncthreads();
        if (sing) break;
        if (p != k)
            for (int j = threadIdx.x; j < r; j += kWG) {
                const double t = E[(int64_t)k * r + j];
                E[(int64_t)k * r + j] = E[(int64_t)p * r + j];
                E[(int64_t)p * r + j] = t;
            }
        __syncthreads();
        const double pk = E[(int64_t)k * r + k];
        for (int i = k + 1 + threadIdx.x; i < r; i += kWG) E[(int64_t)i * r + k] /= pk;
        __syncthreads();
        const int64_t w = r - k - 1;
        for (int64_t q = threadIdx.x; q < w * w; q += kWG) {
            const int i = k + 1 + (int)(q / w), j = k + 1 + (int)(q % w);
            E[(int64_t)i * r + j] -= E[(int64_t)i * r + k] * E[(int64_t)k * r + j];
        }
        __syncthreads();
    }
    if (sing) {
        if (threadIdx.x == 0) atomicOr(flags, 4);
        return;
    }
    // Column a of the inverse: solve (P L U) x = e_a.
    for (int a = threadIdx.x; a < r; a += kWG) {
        double* x = X + (int64_t)a * r;
        for (int i = 0; i < r; ++i) x[i] = (i == a) ? 1.0 : 0.0;
        for (int k = 0; k < r; ++k)
            if (piv[k] != k) {
                const double t = x[k];
                x[k] = x[piv[k]];
                x[piv[k]] = t;
            }
        for (int i = 0; i < r; ++i) {
            double v = x[i];
            for (int j = 0; j < i; ++j) v -= E[(int64_t)i * r + j] * x[j];
            x[i] = v;
        }
        for (int i = r - 1; i >= 0; --i) {
            double v = x[i];
            for (int j = i + 1; j < r; ++j) v -= E[(int64_t)i * r + j] * x[j];
            x[i] = v / E[(int64_t)i * r + i];
        }
    }
}

int lu_inverse(hipStream_t st, int nsys, const int64_t* d_sys_zcol_off, const int64_t* d_e_off,
               double* E, double* Einv, int* d_flags) {
    hipMemsetAsync(d_flags, 0, sizeof(int), st);
    k_lu_inverse<<<nsys, kWG, 0, st>>>(d_sys_zcol_off, d_e_off, E, Einv, d_flags);
    int h = 0;
    hipMemcpyAsync(&h, d_flags, sizeof(int), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusDevice;
    return (h & 4) ? kStatusSingular : kStatusOk;
}

// --------------------------------------------------------- sliced ELL (SELL-64)
// Positions are grouped in slices of 64 (one wavefront); slice s stores the
// entries of its positions column-major, width = longest row of the slice:
// entry k of position p at off[s] + k*64 + (p % 64).  Position p holds row p,
// or row perm[p] when the rows of every 256-row block (one SpMV workgroup)
// are sorted by decreasing length (SELL-C-sigma, C = 64, sigma = 256); the
// sorted order is kept only when it saves at least 1/16 of the stored
// entries (rows of very different lengths side by side, as for tri-quadratic
// hexahedra).  Column indices are stored as 16-bit offsets from the row
// (col - row), which mesh orderings keep small; the copy is not built (all
// outputs NULL, status OK) when an offset falls outside [-32767, 32767].
// Padding entries point at the row itself (offset 0) with a zero value.
// src[q] is the CSR index of entry q (-1 for padding), used to refresh
// values.

__global__ void k_sell_width(int64_t n, const int* __restrict__ rowptr, int* __restrict__ wsz) {
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nsl = (n + 63) / 64;
    if (sl > nsl) return;
    if (sl == nsl) { wsz[sl] = 0; return; }
    int w = 0;
    for (int64_t i = sl * 64; i < min(n, sl * 64 + 64); ++i) w = max(w, rowptr[i + 1] - rowptr[i]);
    wsz[sl] = (int)min((int64_t)w * 64, (int64_t)INT32_MAX);   // saturates: the copy is then refused
}

// Sorted row order of each 256-row block (decreasing length, ties by row) and
// the resulting slice sizes: the first position of a slice holds its longest row.
__global__ __launch_bounds__(kWG) void k_sell_sort(int64_t n, const int* __restrict__ rowptr,
                                                   int* __restrict__ perm, int* __restrict__ wsz) {
    __shared__ int len[kWG];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kWG;
    const int64_t i = r0 + t;
    const int li = i < n ? rowptr[i + 1] - rowptr[i] : -1;
    len[t] = li;
    __syncthreads();
    int rank = 0;
    for (int u = 0; u < kWG; ++u) {
        const int lu = len[u];
        rank += (lu > li) || (lu == li && u < t);
    }
    if (i < n) {
        perm[r0 + rank] = (int)i;
        if (rank % 64 == 0) wsz[(r0 + rank) / 64] = (int)min((int64_t)li * 64, (int64_t)INT32_MAX);
    }
}

__global__ void k_sell_fill(int64_t n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                            const int* __restrict__ off, const int* __restrict__ perm,
                            short* __restrict__ scol, int* __restrict__ src,
                            int* __restrict__ overflow) {
    const int64_t sl = (int64_t)blockIdx.x;     // one block of 64 threads per slice
    const int64_t pos = sl * 64 + threadIdx.x;
    const int64_t i = pos < n && perm ? (int64_t)perm[pos] : pos;
    const int w = (off[sl + 1] - off[sl]) / 64;
    const int base = off[sl] + threadIdx.x;
    const int k0 = i < n ? rowptr[i] : 0;
    const int len = i < n ? rowptr[i + 1] - k0 : 0;
    for (int k = 0; k < w; ++k) {
        const int q = base + k * 64;
        if (k < len) {
            const int64_t d = (int64_t)colind[k0 + k] - i;
            const bool out = d < -32767 || d > 32767;   // symmetric, so A^T fits too
            if (out) *overflow = 1;
            scol[q] = (short)(out ? 0 : d);
            src[q] = k0 + k;
        } else {
            scol[q] = 0;
            src[q] = -1;
        }
    }
}

__global__ void k_sell_vals(int64_t m, const int* __restrict__ src, const double* __restrict__ vals,
                            double* __restrict__ v64, float* __restrict__ v32) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const int k = src[q];
    const double v = k >= 0 ? vals[k] : 0.0;
    if (v64) v64[q] = v;
    if (v32) v32[q] = (float)v;
}

size_t sell_plan_temp_bytes(int64_t n) {
    const int64_t nsl = (n + 63) / 64;
    return 2 * Arena::round((nsl + 1) * sizeof(int)) + scan_temp_bytes(nsl + 1);
}

int sell_plan(hipStream_t st, Arena& ar, int64_t n, const int* rowptr, int* off, int* perm,
              int64_t budget, bool* usable, bool* sorted, int64_t* total, int* wuni) {
    const int64_t nsl = (n + 63) / 64;
    *usable = false;
    *sorted = false;
    *total = 0;
    *wuni = 0;
    const size_t mk = ar.mark();
    int* wsz = ar.temp_n<int>(nsl + 1);
    int* off2 = ar.temp_n<int>(nsl + 1);
    if (!wsz || !off2) {
        ar.release(mk);
        return kStatusNoMem;
    }
    // Slice widths in row order (wsz[nsl] = 0, so off[nsl] is the total).
    k_sell_width<<<blocks_for(nsl + 1), kWG, 0, st>>>(n, rowptr, wsz);
    int64_t h = 0;
    int status = scan_i32(st, ar, wsz, off, nsl + 1, &h);
    // Sorted order within each 256-row block; kept if it stores at least 1/16
    // fewer entries.
    if (status == kStatusOk && nsl > 0) {
        hipMemsetAsync(wsz + nsl, 0, sizeof(int), st);
        k_sell_sort<<<(unsigned)((n + kWG - 1) / kWG), kWG, 0, st>>>(n, rowptr, perm, wsz);
        int64_t h2 = 0;
        status = scan_i32(st, ar, wsz, off2, nsl + 1, &h2);
        if (status == kStatusOk && h2 * 16 <= h * 15) {
            hipMemcpyAsync(off, off2, (nsl + 1) * sizeof(int), hipMemcpyDeviceToDevice, st);
            h = h2;
            *sorted = true;
        }
    }
    if (status == kStatusOk && hipStreamSynchronize(st) != hipSuccess) status = kStatusDevice;
    ar.release(mk);
    if (status != kStatusOk) return status;
    *total = h;
    *usable = nsl > 0 && h < INT32_MAX && h <= budget;
    if (*usable && !*sorted) {
        // Uniform width (every slice as wide as the first): the kernels then
        // compute slice offsets instead of loading them.
        std::vector<int> ho((size_t)nsl + 1);
        if (hipMemcpy(ho.data(), off, (nsl + 1) * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            return kStatusDevice;
        const int w0 = ho[1] - ho[0];
        bool uni = w0 > 0 && w0 % 64 == 0;
        for (int64_t q = 0; uni && q <= nsl; ++q) uni = (int64_t)ho[q] == q * w0;
        if (uni) *wuni = w0 / 64;
    }
    return kStatusOk;
}

int sell_fill_pattern(hipStream_t st, int64_t n, const int* rowptr, const int* colind, const int* off,
                      const int* perm, short* scol, int* src, int* d_flags, bool* usable) {
    const int64_t nsl = (n + 63) / 64;
    int ovf = 0;
    hipMemsetAsync(d_flags, 0, sizeof(int), st);
    if (nsl > 0) k_sell_fill<<<(unsigned)nsl, 64, 0, st>>>(n, rowptr, colind, off, perm, scol, src, d_flags);
    hipMemcpyAsync(&ovf, d_flags, sizeof(int), hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) return kStatusDevice;
    *usable = ovf == 0;
    return kStatusOk;
}

void sell_values(hipStream_t st, int64_t total, const int* src, const double* vals, double* v64,
                 float* v32) {
    if (total > 0) k_sell_vals<<<blocks_for(total), kWG, 0, st>>>(total, src, vals, v64, v32);
}

// ------------------------------------------------- per-block deflation slots
// For the SpMV epilogue that forms Z^T y: row block b (rows [b*RB, (b+1)*RB))
// gets the sorted list of deflation columns its rows reach through Z
// (bb_col[bb_ptr[b] .. bb_ptr[b+1]), one partial-sum slot each); for every
// deflation column a, ab_slot[ab_ptr[a] .. ab_ptr[a+1]) lists its slots in
// increasing block order, so the coarse solve sums them in a fixed order.

__device__ int block_cols(int64_t n, int RB, int64_t blk, const int* __restrict__ zrp,
                          const int* __restrict__ zci, int* cols, bool* over) {
    int nc = 0;
    const int64_t r0 = blk * RB, r1 = min(n, r0 + RB);
    for (int64_t i = r0; i < r1; ++i)
        for (int q = zrp[i]; q < zrp[i + 1]; ++q) {
            const int a = zci[q];
            int t = 0;
            while (t < nc && cols[t] < a) ++t;
            if (t < nc && cols[t] == a) continue;
            if (nc == kBlockColsMax) { *over = true; continue; }
            for (int u = nc; u > t; --u) cols[u] = cols[u - 1];
            cols[t] = a;
            ++nc;
        }
    return nc;
}

__global__ void k_block_cols(int64_t n, int RB, int64_t nblk, const int* __restrict__ zrp,
                             const int* __restrict__ zci, const int* __restrict__ bb_ptr,
                             int* __restrict__ cnt_or_cols, int* __restrict__ flags) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    int cols[kBlockColsMax];
    bool over = false;
    const int nc = block_cols(n, RB, b, zrp, zci, cols, &over);
    if (over) atomicOr(flags, 1);
    if (!bb_ptr) {
        cnt_or_cols[b] = nc;
    } else {
        for (int t = 0; t < nc; ++t) cnt_or_cols[bb_ptr[b] + t] = cols[t];
    }
}

size_t block_slots_temp_bytes(int64_t n, int RB, int R, int64_t cap) {
    const int64_t nblk = (n + RB - 1) / RB;
    return Arena::round((nblk + 1) * sizeof(int)) + scan_temp_bytes(nblk + 1) +
           Arena::round(std::max<int64_t>(cap, 1) * sizeof(int)) + radix_temp_bytes(cap, end_bit_for(R));
}

int build_block_slots(hipStream_t st, Arena& ar, int64_t n, int RB, int R, const int* zrp,
                      const int* zci, int* bb_ptr, int* bb_col, int* ab_ptr, int* ab_slot,
                      int64_t cap, int64_t* nslots, int* d_flags) {
    const int64_t nblk = (n + RB - 1) / RB;
    *nslots = 0;
    const size_t mk = ar.mark();
    int* cnt = ar.temp_n<int>(nblk + 1);
    if (!cnt) return kStatusNoMem;
    hipMemsetAsync(d_flags, 0, sizeof(int), st);
    hipMemsetAsync(cnt + nblk, 0, sizeof(int), st);
    k_block_cols<<<blocks_for(nblk), kWG, 0, st>>>(n, RB, nblk, zrp, zci, nullptr, cnt, d_flags);
    int64_t ns = 0;
    int status = scan_i32(st, ar, cnt, bb_ptr, nblk + 1, &ns);
    if (status == kStatusOk) {
        int fl = 0;
        hipMemcpyAsync(&fl, d_flags, sizeof(int), hipMemcpyDeviceToHost, st);
        if (hipStreamSynchronize(st) != hipSuccess) status = kStatusDevice;
        else if (fl || ns > cap) status = kStatusInval;   // some block reaches too many columns
    }
    if (status == kStatusOk) {
        int* keys_out = ar.temp_n<int>(ns);
        if (!keys_out) {
            status = kStatusNoMem;
        } else {
            k_block_cols<<<blocks_for(nblk), kWG, 0, st>>>(n, RB, nblk, zrp, zci, bb_ptr, bb_col, d_flags);
            status = radix_sort_pairs(st, ar, ns, bb_col, end_bit_for(R), keys_out, ab_slot);
            if (status == kStatusOk) {
                k_bounds<<<blocks_for(ns + 1), kWG, 0, st>>>(ns, R, keys_out, ab_ptr);
                if (hipStreamSynchronize(st) != hipSuccess) status = kStatusDevice;
            }
        }
    }
    ar.release(mk);
    if (status == kStatusOk) *nslots = ns;
    return status;
}

// ---------------------------------------------- single-entry row copies (ELL-1)
// c1[i] = the only column of row i (>= 0), -1 for an empty row, -2 for a row
// with several entries (the CSR is used for those); v1[i] its value.  Lets the
// streaming kernels read one coalesced (column, value) pair per row.
__global__ void k_ell1(int64_t n, const int* __restrict__ rp, const int* __restrict__ ci,
                       const double* __restrict__ v, int* __restrict__ c1, double* __restrict__ v1,
                       float* __restrict__ v1f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int q0 = rp[i], q1 = rp[i + 1];
    int c = -1;
    double val = 0.0;
    if (q1 - q0 == 1) {
        c = ci[q0];
        val = v[q0];
    } else if (q1 - q0 > 1) {
        c = -2;
    }
    if (c1) c1[i] = c;
    v1[i] = val;
    if (v1f) v1f[i] = (float)val;
}

void ell1_build(hipStream_t st, int64_t n, const int* rp, const int* ci, const double* v, int* c1,
                double* v1, float* v1f) {
    if (n > 0) k_ell1<<<blocks_for(n), kWG, 0, st>>>(n, rp, ci, v, c1, v1, v1f);
}

// Two-entry row copies (ELL-2, interleaved per row): c2[2i], c2[2i+1] = the
// columns of row i's first and second entries (-1 where absent, value 0);
// rows with three or more entries get c2[2i] = -2 and zero values (the CSR is
// used for those).  With an indicator deflation basis on a 2-D mesh, A Z has
// at most two entries per row except near subdomain corners.
__global__ void k_ell2(int64_t n, const int* __restrict__ rp, const int* __restrict__ ci,
                       const double* __restrict__ v, int* __restrict__ c2, double* __restrict__ v2,
                       float* __restrict__ v2f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int q0 = rp[i], q1 = rp[i + 1];
    int ca = -1, cb = -1;
    double va = 0.0, vb = 0.0;
    if (q1 - q0 > 2) {
        ca = -2;
    } else {
        if (q1 - q0 >= 1) {
            ca = ci[q0];
            va = v[q0];
        }
        if (q1 - q0 == 2) {
            cb = ci[q0 + 1];
            vb = v[q0 + 1];
        }
    }
    if (c2) {
        c2[2 * i] = ca;
        c2[2 * i + 1] = cb;
    }
    v2[2 * i] = va;
    v2[2 * i + 1] = vb;
    if (v2f) {
        v2f[2 * i] = (float)va;
        v2f[2 * i + 1] = (float)vb;
    }
}

void ell2_build(hipStream_t st, int64_t n, const int* rp, const int* ci, const double* v, int* c2,
                double* v2, float* v2f) {
    if (n > 0) k_ell2<<<blocks_for(n), kWG, 0, st>>>(n, rp, ci, v, c2, v2, v2f);
}

// Inverse permutation: pos[perm[q]] = q.
__global__ void k_invperm(int64_t m, const int* __restrict__ perm, int* __restrict__ pos) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) pos[perm[q]] = (int)q;
}

void invperm(hipStream_t st, int64_t m, const int* perm, int* pos) {
    if (m > 0) k_invperm<<<blocks_for(m), kWG, 0, st>>>(m, perm, pos);
}

// ------------------------------------------------------------ small kernels

__global__ void k_to_f32(int64_t n, const double* __restrict__ s, float* __restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

void to_f32(hipStream_t st, int64_t n, const double* src, float* dst) {
    if (n > 0) k_to_f32<<<blocks_for(n), kWG, 0, st>>>(n, src, dst);
}

// dL/dA_ij = -lambda_i x_j on the pattern of A.
__global__ void k_grad_vals(int64_t n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                            const double* __restrict__ lam, const double* __restrict__ x,
                            double* __restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double li = lam[i];
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) g[k] = -li * x[colind[k]];
}

void grad_vals(hipStream_t st, int64_t n, const int* rowptr, const int* colind, const double* lam,
               const double* x, double* g) {
    k_grad_vals<<<blocks_for(n), kWG, 0, st>>>(n, rowptr, colind, lam, x, g);
}

__global__ void k_max_row(int R, const int* __restrict__ rp, int* __restrict__ out) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < R) atomicMax(out, rp[a + 1] - rp[a]);
}

int zt_max_row(hipStream_t st, int R, const int* ztrp, int* d_tmp) {
    hipMemsetAsync(d_tmp, 0, sizeof(int), st);
    if (R > 0) k_max_row<<<blocks_for(R), kWG, 0, st>>>(R, ztrp, d_tmp);
    int h = 0;
    hipMemcpyAsync(&h, d_tmp, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    return h;
}

GM_DEBUG_ACCESSOR(dbg_take_setup)

}  // namespace gm
