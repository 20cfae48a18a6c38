// Persistent batched deflated GMRES(m): many independent systems in one launch.
//
// Each workgroup takes systems from an atomic ticket queue (systems ordered by
// decreasing work, so the largest start first) and runs the whole solve of a
// system -- every restart cycle -- with workgroup-local barriers only, so no
// workgroup ever waits for another and every workgroup exits once the queue is
// empty.  Per system: convergence state, iteration count, status and device
// timestamps (start/end of its solve).
//
// The arithmetic per system is that of the single-system path (arXiv
// 1906.04051, Sec. 3.2-3.3): deflated operator P A, Arnoldi with CGS2, plane
// rotations and |gamma_{k+1}| (eq. res), x_m = x_0 + V_m y_m, restarts from x_m
// with the true residual test (eq. relative), and the final coarse correction.
#include "internal.hpp"

namespace gm {

// Sum of v over the workgroup (fixed order), valid in every thread.
template <int WGS>
__device__ __forceinline__ double bsum(double v, double* red) {
    constexpr int NW = WGS / kWave;
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Lane layout of the passes: T consecutive lanes share one row; lane `sub`
// owns basis columns k = sub, sub + T, ... (JT = MB / T of them), so each lane
// keeps JT basis values and dot accumulators in registers.
template <int T>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Workgroup sums of acc[q] (column sub + q*T) into out[k] for k < nv and of
// accn into out[nv].  Fixed order: butterfly over lanes of equal `sub`, then
// waves in order.
template <int WGS, int MB, int T>
__device__ __forceinline__ void bsum_cols(const double (&acc)[MB / T], double accn, int nv,
                                          double (*red)[MB + 1], double* out) {
    constexpr int NW = WGS / kWave;
    constexpr int JT = MB / T;
    const int w = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
    const int sub = ln & (T - 1);
#pragma unroll
    for (int q = 0; q < JT; ++q)
        if (q * T < nv) {
            double t = acc[q];
#pragma unroll
            for (int o = kWave / 2; o >= T; o >>= 1) t += __shfl_xor(t, o, kWave);
            const int k = sub + q * T;
            if (ln < T && k < nv) red[w][k] = t;
        }
    {
        const double t = wave_sum(accn);
        if (ln == 0) red[w][MB] = t;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < nv || t == MB) {
        double s = red[0][t];
#pragma unroll
        for (int q = 1; q < NW; ++q) s += red[q][t];
        out[t < nv ? t : nv] = s;
    }
    __syncthreads();
}

template <int WGS, int L, int MB>
__global__ __launch_bounds__(WGS) void k_batched(BatchArgs a) {
    constexpr int NW = WGS / kWave;
    constexpr int kRows = WGS / L;
    constexpr int T = MB / 8;            // lanes per row in the passes (8 columns per lane)
    constexpr int JT = MB / T;
    constexpr int PR = WGS / T;          // rows per pass iteration
    __shared__ double red[NW][MB + 1];
    __shared__ double sred[NW];
    __shared__ double Hs[(MB + 1) * MB];
    __shared__ double cs[MB], sn[MB], g[MB + 1], vscale[MB + 1];
    __shared__ double h1[MB + 1], h2[MB + 1], coef[MB + 1], tvec[kMaxR], svec[kMaxR];
    __shared__ int s_sys;
    __shared__ int s_flag;

    const int m = a.m;
    const int lane = threadIdx.x & (L - 1);
    for (;;) {
        if (threadIdx.x == 0) {
            const int t = atomicAdd(a.ticket, 1);
            s_sys = (t < a.nsys) ? a.order[t] : -1;
        }
        __syncthreads();
        const int sys = s_sys;
        __syncthreads();
        if (sys < 0) break;

        const int64_t r0 = a.row_off[sys];
        const int n = (int)(a.row_off[sys + 1] - r0);
        const int64_t c0 = a.zcol_off[sys];
        const int R = (int)(a.zcol_off[sys + 1] - c0);
        const double* Einv = a.Einv + a.e_off[sys];
        double* V = a.V + a.v_off[sys];
        const int64_t ldv = n;
        double* y = a.W + 3 * r0;
        double* w = y + n;
        double* rr = w + n;
        double* x = a.x + r0;
        const double* b = a.b + r0;
        uint64_t t_start = wall_clock64();

        // Residual r = b - A x of the current x (global row/col indices).
        auto residual = [&](double* out) -> double {
            double acc = 0;
            for (int row = threadIdx.x / L; row < n; row += kRows) {
                const int64_t gi = r0 + row;
                const int k0 = a.rowptr[gi], k1 = a.rowptr[gi + 1];
                double s = 0;
                for (int k = k0 + lane; k < k1; k += L) s += a.vals[k] * x[a.colind[k] - r0];
#pragma unroll
                for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
                if (lane == 0) {
                    const double ri = b[row] - s;
                    out[row] = ri;
                    acc += ri * ri;
                }
            }
            __syncthreads();
            return bsum<WGS>(acc, sred);
        };
        // svec = E^{-1} Z^T vec  (one wave per row of Z^T, then a small matvec).
        auto coarse = [&](const double* vec) {
            if (R == 0) return;
            const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
            for (int c = wv; c < R; c += NW) {
                const int q0 = a.ztrp[c0 + c], q1 = a.ztrp[c0 + c + 1];
                double s = 0;
                for (int q = q0 + ln; q < q1; q += kWave) s += a.ztv[q] * vec[a.ztci[q] - r0];
                s = wave_sum(s);
                if (ln == 0) tvec[c] = s;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < R; i += WGS) {
                double s = 0;
                for (int c = 0; c < R; ++c) s += Einv[(int64_t)c * R + i] * tvec[c];
                svec[i] = s;
            }
            __syncthreads();
        };
        auto deflate_row = [&](int64_t gi, double v) -> double {
            for (int q = a.azrp[gi]; q < a.azrp[gi + 1]; ++q) v -= a.azv[q] * svec[a.azci[q] - c0];
            return v;
        };

        // x0
        for (int i = threadIdx.x; i < n; i += WGS) x[i] = a.x0 ? a.x0[r0 + i] : 0.0;
        __syncthreads();
        const double rho0 = sqrt(residual(rr));
        const double target = a.rtol * rho0;
        int64_t its = 0;
        int cycles = 0;
        int status = kStatusOk;
        double beta = 0.0;
        bool first = true;
        for (;;) {
            if (!first) {
                residual(rr);
            }
            first = false;
            if (rho0 == 0.0) { beta = 0.0; break; }
            coarse(rr);
            double accn = 0;
            for (int i = threadIdx.x; i < n; i += WGS) {
                const double p = deflate_row(r0 + i, rr[i]);
                V[i] = p;
                accn += p * p;
            }
            beta = sqrt(bsum<WGS>(accn, sred));
            if (!isfinite(beta)) { status = kStatusNonFinite; break; }
            if (beta <= target) { status = kStatusOk; break; }
            if (its >= a.max_iters) { status = kStatusMaxIter; break; }
            ++cycles;
            if (threadIdx.x == 0) {
                g[0] = beta;
                for (int i = 1; i <= m; ++i) g[i] = 0.0;
                vscale[0] = 1.0 / beta;
            }
            __syncthreads();
            int kk = 0;
            for (int j = 0; j < m && its < a.max_iters; ++j) {
                const int nv = j + 1;
                const double* vj = V + (int64_t)j * ldv;
                const double sj = vscale[j];
                // y = A v_j (normalised)
                for (int row = threadIdx.x / L; row < n; row += kRows) {
                    const int64_t gi = r0 + row;
                    const int k0 = a.rowptr[gi], k1 = a.rowptr[gi + 1];
                    double s = 0;
                    for (int k = k0 + lane; k < k1; k += L) s += a.vals[k] * vj[a.colind[k] - r0];
#pragma unroll
                    for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
                    if (lane == 0) y[row] = s * sj;
                }
                __syncthreads();
                coarse(y);
                // pass 1: w = P y; dots with stored basis; ||w||^2
                const int sub = threadIdx.x & (T - 1);
                double acc[JT];
#pragma unroll
                for (int q = 0; q < JT; ++q) acc[q] = 0;
                accn = 0;
                for (int i = threadIdx.x / T; i < n; i += PR) {
                    double vv[JT];
#pragma unroll
                    for (int q = 0; q < JT; ++q)
                        if (sub + q * T < nv) vv[q] = V[(int64_t)(sub + q * T) * ldv + i];
                    const double wi = (R > 0) ? deflate_row(r0 + i, y[i]) : y[i];
                    if (sub == 0) {
                        w[i] = wi;
                        accn += wi * wi;
                    }
#pragma unroll
                    for (int q = 0; q < JT; ++q)
                        if (sub + q * T < nv) acc[q] += vv[q] * wi;
                }
                bsum_cols<WGS, MB, T>(acc, accn, nv, red, h1);
                const double wpre2 = h1[nv];
                for (int k = threadIdx.x; k < nv; k += WGS) {
                    h1[k] *= vscale[k];
                    coef[k] = h1[k] * vscale[k];
                }
                __syncthreads();
                // pass 2
#pragma unroll
                for (int q = 0; q < JT; ++q) acc[q] = 0;
                accn = 0;
                for (int i = threadIdx.x / T; i < n; i += PR) {
                    double vv[JT];
#pragma unroll
                    for (int q = 0; q < JT; ++q)
                        if (sub + q * T < nv) vv[q] = V[(int64_t)(sub + q * T) * ldv + i];
                    double u = 0;
#pragma unroll
                    for (int q = 0; q < JT; ++q)
                        if (sub + q * T < nv) u += vv[q] * coef[sub + q * T];
                    const double wi = w[i] - gsum<T>(u);
                    if (sub == 0) {
                        w[i] = wi;
                        accn += wi * wi;
                    }
#pragma unroll
                    for (int q = 0; q < JT; ++q)
                        if (sub + q * T < nv) acc[q] += vv[q] * wi;
                }
                bsum_cols<WGS, MB, T>(acc, accn, nv, red, h2);
                for (int k = threadIdx.x; k < nv; k += WGS) {
                    h2[k] *= vscale[k];
                    coef[k] = h2[k] * vscale[k];
                }
                __syncthreads();
                // pass 3: new basis column
                double* vout = V + (int64_t)nv * ldv;
                accn = 0;
                for (int i = threadIdx.x / T; i < n; i += PR) {
                    double u = 0;
#pragma unroll
                    for (int q = 0; q < JT; ++q)
                        if (sub + q * T < nv) u += V[(int64_t)(sub + q * T) * ldv + i] * coef[sub + q * T];
                    const double wi = w[i] - gsum<T>(u);
                    if (sub == 0) {
                        vout[i] = wi;
                        accn += wi * wi;
                    }
                }
                const double hn = sqrt(bsum<WGS>(accn, sred));
                if (threadIdx.x == 0) {
                    const int bd = !(hn > 2.220446049250313e-16 * sqrt(wpre2));
                    double a0 = h1[0] + h2[0];
                    for (int i = 0; i < j; ++i) {
                        const double c = cs[i], sv = sn[i], bb = h1[i + 1] + h2[i + 1];
                        Hs[i * MB + j] = c * a0 + sv * bb;
                        a0 = -sv * a0 + c * bb;
                    }
                    double rho = hypot(a0, hn);
                    if (hn == 0.0) { cs[j] = 1.0; sn[j] = 0.0; rho = a0; }
                    else { cs[j] = a0 / rho; sn[j] = hn / rho; }
                    Hs[j * MB + j] = rho;
                    g[j + 1] = -sn[j] * g[j];
                    g[j] = cs[j] * g[j];
                    vscale[nv] = bd ? 0.0 : 1.0 / hn;
                    s_flag = (fabs(g[j + 1]) <= target || bd) ? 1 : 0;
                }
                __syncthreads();
                ++its;
                kk = nv;
                if (s_flag) break;
            }
            // y_k = R^{-1} g (column-oriented, all threads), x += V_k y_k
            for (int i = threadIdx.x; i < kk; i += WGS) h2[i] = g[i];
            __syncthreads();
            for (int i = kk - 1; i >= 0; --i) {
                const double yi = h2[i] / Hs[i * MB + i];
                for (int l = threadIdx.x; l < i; l += WGS) h2[l] -= Hs[l * MB + i] * yi;
                if (threadIdx.x == 0) coef[i] = yi * vscale[i];
                __syncthreads();
            }
            for (int i = threadIdx.x; i < n; i += WGS) {
                double acc = 0;
                for (int t = 0; t < kk; ++t) acc += V[(int64_t)t * ldv + i] * coef[t];
                x[i] += acc;
            }
            __syncthreads();
        }
        // Final coarse correction x = x_hat + Z E^{-1} Z^T (b - A x_hat).
        if (rho0 > 0.0 && R > 0) {
            for (int i = threadIdx.x; i < n; i += WGS) {
                double v = x[i];
                for (int q = a.zrp[r0 + i]; q < a.zrp[r0 + i + 1]; ++q) v += a.zv[q] * svec[a.zci[q] - c0];
                x[i] = v;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t t_end = wall_clock64();
            a.out_i[3 * sys + 0] = its;
            a.out_i[3 * sys + 1] = cycles;
            a.out_i[3 * sys + 2] = status;
            a.out_d[4 * sys + 0] = rho0;
            a.out_d[4 * sys + 1] = rho0 > 0.0 ? beta / rho0 : 0.0;
            a.out_d[4 * sys + 2] = (double)t_start;
            a.out_d[4 * sys + 3] = (double)t_end;
        }
        __syncthreads();
    }
}

template <int WGS, int MB>
static void launch_l(const BatchArgs& a, int nwg) {
    switch (a.L) {
        case 4: k_batched<WGS, 4, MB><<<nwg, WGS, 0, a.st>>>(a); break;
        case 8: k_batched<WGS, 8, MB><<<nwg, WGS, 0, a.st>>>(a); break;
        case 16: k_batched<WGS, 16, MB><<<nwg, WGS, 0, a.st>>>(a); break;
        default: k_batched<WGS, 32, MB><<<nwg, WGS, 0, a.st>>>(a); break;
    }
}

// Per-system ||b - A x||^2 (one workgroup per system, fixed order).
__global__ __launch_bounds__(kWG) void k_seg_resid(int nsys, const int64_t* __restrict__ row_off,
                                                   const int* __restrict__ rowptr,
                                                   const int* __restrict__ colind,
                                                   const double* __restrict__ vals,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ out) {
    __shared__ double red[kWG / kWave];
    const int s = blockIdx.x;
    double acc = 0;
    for (int64_t i = row_off[s] + threadIdx.x; i < row_off[s + 1]; i += kWG) {
        double v = b[i];
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) v -= vals[k] * x[colind[k]];
        acc += v * v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[s] = acc;
}

void launch_seg_resid(hipStream_t st, int nsys, const int64_t* row_off, const int* rowptr,
                      const int* colind, const double* vals, const double* x, const double* b,
                      double* out) {
    k_seg_resid<<<nsys, kWG, 0, st>>>(nsys, row_off, rowptr, colind, vals, x, b, out);
}

void launch_batched(const BatchArgs& a, int nwg) {
    const bool big = a.m > 32;
    switch (a.wg) {
        case 512:
            if (big) launch_l<512, 64>(a, nwg); else launch_l<512, 32>(a, nwg);
            break;
        case 1024:
            if (big) launch_l<1024, 64>(a, nwg); else launch_l<1024, 32>(a, nwg);
            break;
        default:
            if (big) launch_l<256, 64>(a, nwg); else launch_l<256, 32>(a, nwg);
            break;
    }
}

}  // namespace gm
