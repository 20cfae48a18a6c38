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

// Lane layout of the passes: T consecutive lanes share one row pair; lane
// `sub` owns basis columns k = sub, sub + T, ... (JT = 8 of them), so each
// lane keeps JT basis values and dot accumulators in registers.  T is chosen
// per Arnoldi step (the smallest power of two with 8 T >= nv) and is the same
// in every lane, so the shuffles below stay inside aligned groups of T lanes.
__device__ __forceinline__ double gsum(double v, int T) {
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Workgroup sums of acc[q] (column sub + q*T) into out[k] for k < nv and of
// accn into out[nv].  Fixed order: butterfly over lanes of equal `sub`, then
// waves in order.
template <int WGS, int MB, int JT>
__device__ __forceinline__ void bsum_cols(const double (&acc)[JT], double accn, int nv, int T,
                                          double (*red)[MB + 1], double* out) {
    constexpr int NW = WGS / kWave;
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

// 16-byte loads and stores of row pairs (the per-system regions start at even
// offsets and have an even leading dimension).
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ void st2(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }

constexpr int kZf = 16;   // deflation columns per system that the SpMV's fused Z^T y holds per lane

template <int WGS, int L, int MB>
__global__ __launch_bounds__(WGS) void k_batched(BatchArgs a) {
    constexpr int NW = WGS / kWave;
    constexpr int kRows = WGS / L;       // rows per SpMV round (L lanes per row)
    constexpr int JT = 8;                // basis columns per lane in the sweeps
    constexpr int U = 2;                 // sweep rounds whose loads are in flight together
    __shared__ double red[NW][MB + 1];
    __shared__ double sred[NW];
    __shared__ double zred[NW][kZf];
    __shared__ double Hs[(MB + 1) * MB];
    __shared__ double cs[MB], sn[MB], g[MB + 1], vscale[MB + 1];
    __shared__ double h1[MB + 1], h2[MB + 1], coef[MB + 1], tvec[kMaxR], svec[kMaxR];
    __shared__ double Hr[(MB + 1) * MB];   // unrotated Hessenberg of the cycle
    __shared__ double cc[MB + 1];          // next step's (H h2) coefficients of the stored columns
    __shared__ double lag[2];              // h2 of the last column, 1 / hn
    __shared__ int s_sys;
    __shared__ int s_flag;

    const int m = a.m;
    const int lane = threadIdx.x & (L - 1);
    const int wv = threadIdx.x / kWave, ln = threadIdx.x & (kWave - 1);
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
        const int np = (n + 1) / 2;              // row pairs
        const int64_t ld = 2 * (int64_t)np;      // leading dimension of the system's regions
        const int64_t c0 = a.zcol_off[sys];
        const int R = (int)(a.zcol_off[sys + 1] - c0);
        const bool fz = R > 0 && R <= kZf;       // Z^T y fused into the SpMV
        const double* Einv = a.Einv + a.e_off[sys];
        double* V = a.V + a.v_off[sys];
        double* y = a.W + a.w_off[sys];
        double* w = y + ld;
        double* rr = w + ld;
        double* x = a.x + r0;
        const double* b = a.b + r0;
        uint64_t t_start = wall_clock64();

        // svec = E^{-1} tvec (tvec = Z^T vec, local deflation columns).
        auto coarse_solve = [&]() {
            for (int i = threadIdx.x; i < R; i += WGS) {
                double s = 0;
                for (int c = 0; c < R; ++c) s += Einv[(int64_t)c * R + i] * tvec[c];
                svec[i] = s;
            }
            __syncthreads();
        };
        // tvec = Z^T vec one wavefront per row of Z^T (when not fused).
        auto zt_waves = [&](const double* vec) {
            for (int c = wv; c < R; c += NW) {
                const int q0 = a.ztrp[c0 + c], q1 = a.ztrp[c0 + c + 1];
                double s = 0;
                for (int q = q0 + ln; q < q1; q += kWave) s += a.ztv[q] * vec[a.ztci[q] - r0];
                s = wave_sum(s);
                if (ln == 0) tvec[c] = s;
            }
            __syncthreads();
        };
        // Per-lane Z^T partials of one row value, summed over the workgroup
        // in fixed order by zt_finish.
        auto zt_add = [&](double (&zacc)[kZf], int64_t gi, double v, int zc, double zv) {
            if (zc >= 0) {
                const double t = zv * v;
#pragma unroll
                for (int c = 0; c < kZf; ++c) zacc[c] += (zc - (int)c0 == c) ? t : 0.0;
            } else if (zc == -2) {
                for (int q = a.zrp[gi]; q < a.zrp[gi + 1]; ++q) {
                    const int cz = a.zci[q] - (int)c0;
                    const double t = a.zv[q] * v;
#pragma unroll
                    for (int c = 0; c < kZf; ++c) zacc[c] += (cz == c) ? t : 0.0;
                }
            }
        };
        auto zt_finish = [&](double (&zacc)[kZf]) {
#pragma unroll
            for (int c = 0; c < kZf; ++c) {
                const double t = wave_sum(zacc[c]);
                if (ln == 0) zred[wv][c] = t;
            }
            __syncthreads();
            if (threadIdx.x < R) {
                double t = zred[0][threadIdx.x];
#pragma unroll
                for (int q = 1; q < NW; ++q) t += zred[q][threadIdx.x];
                tvec[threadIdx.x] = t;
            }
            __syncthreads();
        };
        // out = scale * A xin (mode 0) or out = b - A xin (residual), two rows
        // per lane group in flight; with fz also tvec = Z^T out.  Returns the
        // workgroup sum of out^2 (residual mode).
        auto spmv = [&](const double* xin, double scale, bool resid, double* out) -> double {
            double zacc[kZf];
#pragma unroll
            for (int c = 0; c < kZf; ++c) zacc[c] = 0.0;
            double acc = 0;
            if (a.sell_col) {
                // Sliced ELL: one wavefront per 64-row slice overlapping the
                // system (rows of other systems in an edge slice are skipped);
                // the entries of a chunk, the row's b value and its Z row copy
                // are loaded before any gather (two memory round trips per
                // slice).
                constexpr int CH = 16;
                const int64_t sl0 = r0 / kWave, sl1 = (r0 + n + kWave - 1) / kWave;
                for (int64_t sl = sl0 + wv; sl < sl1; sl += NW) {
                    const int64_t gi = sl * kWave + ln;
                    const bool ok = gi >= r0 && gi < r0 + n;
                    int q0, w;
                    if (a.sell_wuni > 0) {
                        q0 = (int)(sl * a.sell_wuni * kWave);
                        w = a.sell_wuni;
                    } else {
                        q0 = __builtin_amdgcn_readfirstlane(a.sell_off[sl]);
                        w = (__builtin_amdgcn_readfirstlane(a.sell_off[sl + 1]) - q0) / kWave;
                    }
                    const double bvv = (resid && ok) ? b[gi - r0] : 0.0;
                    const int zc = (fz && ok) ? a.zc1[gi] : -1;
                    const double zv = (fz && ok) ? a.zv1[gi] : 0.0;
                    // Rows outside the system gather from the system's own first row.
                    const double* xr = xin + (ok ? gi - r0 : 0);
                    double s = 0;
                    for (int k0 = 0; k0 < w; k0 += CH) {
                        short cc[CH];
                        double vv[CH];
#pragma unroll
                        for (int k = 0; k < CH; ++k) {
                            const int qk = q0 + min(k0 + k, w - 1) * kWave + ln;
                            cc[k] = a.sell_col[qk];
                            vv[k] = a.sell_val[qk];
                        }
                        double xv[CH];
#pragma unroll
                        for (int k = 0; k < CH; ++k) {
                            GM_DCHECK(!ok || k0 + k >= w || (gi - r0 + cc[k] >= 0 && gi - r0 + cc[k] < n),
                                      kDbgBatchCol);
                            xv[k] = xr[ok ? (int)cc[k] : 0];
                        }
#pragma unroll
                        for (int k = 0; k < CH; ++k) s += (ok && k0 + k < w) ? vv[k] * xv[k] : 0.0;
                    }
                    if (ok) {
                        const double v = resid ? bvv - s : s * scale;
                        out[gi - r0] = v;
                        if (resid) acc += v * v;
                        if (fz) zt_add(zacc, gi, v, zc, zv);
                    }
                }
                __syncthreads();
                if (fz) zt_finish(zacc);
                else if (R > 0) zt_waves(out);
                return resid ? bsum<WGS>(acc, sred) : 0.0;
            }
            for (int row0 = threadIdx.x / L; row0 < n; row0 += 2 * kRows) {
                int k0[2], k1[2];
                double bv[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int row = row0 + u * kRows;
                    const bool ok = row < n;
                    k0[u] = ok ? a.rowptr[r0 + row] : 0;
                    k1[u] = ok ? a.rowptr[r0 + row + 1] : 0;
                    bv[u] = (resid && ok) ? b[row] : 0.0;
                }
                double sacc[2] = {0.0, 0.0};
                for (int e = lane;; e += L) {
                    const bool ok0 = k0[0] + e < k1[0], ok1 = k0[1] + e < k1[1];
                    if (!ok0 && !ok1) break;
                    const int col0 = ok0 ? a.colind[k0[0] + e] : (int)r0;
                    const int col1 = ok1 ? a.colind[k0[1] + e] : (int)r0;
                    const double v0 = ok0 ? a.vals[k0[0] + e] : 0.0;
                    const double v1 = ok1 ? a.vals[k0[1] + e] : 0.0;
                    GM_DCHECK(col0 - r0 >= 0 && col0 - r0 < n && col1 - r0 >= 0 && col1 - r0 < n, kDbgBatchCol);
                    sacc[0] += v0 * xin[col0 - r0];
                    sacc[1] += v1 * xin[col1 - r0];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
#pragma unroll
                    for (int o = L / 2; o > 0; o >>= 1) sacc[u] += __shfl_xor(sacc[u], o, L);
                    const int row = row0 + u * kRows;
                    if (lane == 0 && row < n) {
                        const double v = resid ? bv[u] - sacc[u] : sacc[u] * scale;
                        out[row] = v;
                        if (resid) acc += v * v;
                        if (fz) zt_add(zacc, r0 + row, v, a.zc1[r0 + row], a.zv1[r0 + row]);
                    }
                }
            }
            __syncthreads();
            if (fz) zt_finish(zacc);
            else if (R > 0) zt_waves(out);
            return resid ? bsum<WGS>(acc, sred) : 0.0;
        };
        // v - (A Z)_row svec for local row i < n from the row's two-entry copy
        // (c2, v2; c2.x == -2: three or more entries, read from the CSR copy).
        auto deflate_pre = [&](int i, double v, int2 c2, double2 v2) -> double {
            if (c2.x >= 0) {
                v -= v2.x * svec[c2.x - c0];
                if (c2.y >= 0) v -= v2.y * svec[c2.y - c0];
            } else if (c2.x == -2) {
                const int64_t gi = r0 + i;
                for (int q = a.azrp[gi]; q < a.azrp[gi + 1]; ++q) v -= a.azv[q] * svec[a.azci[q] - c0];
            }
            return v;
        };
        auto deflate_row = [&](int i, double v) -> double {
            const int64_t gi = r0 + i;
            const int2 c2 = *reinterpret_cast<const int2*>(a.az2c + 2 * gi);
            const double2 v2 = c2.x >= 0 ? ld2(a.az2v + 2 * gi) : make_double2(0.0, 0.0);
            return deflate_pre(i, v, c2, v2);
        };
        // vec -= (A Z) svec over the system's rows, in place; four rows per
        // thread with their loads issued together (the sweeps then read a
        // projected vector and wait on one round trip per row pair).
        auto deflate_vec = [&](double* vec) {
            constexpr int DU = 4;
            for (int i0 = threadIdx.x; i0 < n; i0 += DU * WGS) {
                double v[DU];
                int2 c2[DU];
                double2 v2[DU];
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const int i = i0 + u * WGS;
                    const bool ok = i < n;
                    const int64_t gi = r0 + (ok ? i : 0);
                    v[u] = ok ? vec[i] : 0.0;
                    c2[u] = ok ? *reinterpret_cast<const int2*>(a.az2c + 2 * gi) : make_int2(-1, -1);
                    v2[u] = ok ? ld2(a.az2v + 2 * gi) : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const int i = i0 + u * WGS;
                    if (i < n) vec[i] = deflate_pre(i, v[u], c2[u], v2[u]);
                }
            }
            __syncthreads();
        };

        // x0
        for (int i = threadIdx.x; i < n; i += WGS) x[i] = a.x0 ? a.x0[r0 + i] : 0.0;
        __syncthreads();
        const double rho0 = sqrt(spmv(x, 1.0, true, rr));
        const double target = a.rtol * rho0;
        int64_t its = 0;
        int cycles = 0;
        int status = kStatusOk;
        double beta = 0.0;
        bool first = true;
        for (;;) {
            if (!first) spmv(x, 1.0, true, rr);
            first = false;
            if (rho0 == 0.0) { beta = 0.0; break; }
            if (R > 0) coarse_solve();
            double accn = 0;
            for (int i = threadIdx.x; i < n; i += WGS) {
                const double p = R > 0 ? deflate_row(i, rr[i]) : rr[i];
                V[i] = p;
                accn += p * p;
            }
            beta = sqrt(bsum<WGS>(accn, sred));
            if (!isfinite(beta)) { status = kStatusNonFinite; break; }
            if (beta <= target) { status = kStatusOk; break; }
            if (its >= a.max_iters) { status = kStatusMaxIter; break; }
            // A system with a continuation plan leaves at the first restart
            // past its step limit, with x = x_hat + Z E^{-1} Z^T r (below).
            if (a.hand && a.hand[sys] > 0 && its >= a.hand[sys]) { status = kStatusHandoff; break; }
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
                // Lanes per row pair of this step's sweeps (more row pairs in
                // flight while the basis is short) and row pairs per round.
                const int T = nv <= 8 ? 1 : (nv <= 16 ? 2 : (nv <= 32 ? 4 : 8));
                const int PR = WGS / T;
                const int sub = threadIdx.x & (T - 1);
                // Two sweeps per step (CGS2 with lagged normalisation): step j
                // >= 1 runs the SpMV on the previous step's once-projected w1
                // (unnormalised) and sweep A forms, in one pass over v_0..v_{j-1},
                //   w2 = w1 - V h2          (second projection; stored as v_j),
                //   w  = (P A w1 - V c - w2 h2_{j-1}) / hn = P A v_j,
                // with c = H h2 (the Arnoldi relation P A V = V H, rows < j) and
                // hn = ||w2|| estimated as sqrt(||w1||^2 - ||h2||^2); then its
                // dots with v_0..v_j.  Sweep B (pass 2) projects once more.
                // Step 0: y = A v_0 and pass 1 as usual.
                double wpre2;
                if (j == 0) {
                    spmv(V, vscale[0], false, y);
                    if (R > 0) {
                        coarse_solve();
                        deflate_vec(y);   // y = P A v_0
                    }
                    // pass 1: w = P y; dots with v_0; ||w||^2
                    double acc[JT];
#pragma unroll
                    for (int q = 0; q < JT; ++q) acc[q] = 0;
                    accn = 0;
                    for (int p0 = threadIdx.x / T; p0 < np; p0 += U * PR) {
                        double2 vv[U][JT], yy[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int pp = p0 + u * PR;
                            const bool ok = pp < np;
#pragma unroll
                            for (int q = 0; q < JT; ++q) {
                                const int k = sub + q * T;
                                vv[u][q] = (ok && k < nv) ? ld2(V + (int64_t)k * ld + 2 * pp) : make_double2(0.0, 0.0);
                            }
                            yy[u] = ok ? ld2(y + 2 * pp) : make_double2(0.0, 0.0);
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int pp = p0 + u * PR;
                            if (pp >= np) continue;
                            const int i = 2 * pp;
                            double2 wv2 = yy[u];
                            if (i + 1 >= n) wv2.y = 0.0;
                            if (sub == 0) {
                                st2(w + i, wv2);
                                accn += wv2.x * wv2.x + wv2.y * wv2.y;
                            }
#pragma unroll
                            for (int q = 0; q < JT; ++q) acc[q] += vv[u][q].x * wv2.x + vv[u][q].y * wv2.y;
                        }
                    }
                    bsum_cols<WGS, MB, JT>(acc, accn, nv, T, red, h1);
                    wpre2 = h1[nv];
                } else {
                    spmv(w, 1.0, false, y);
                    if (R > 0) {
                        coarse_solve();
                        deflate_vec(y);   // y = P A w1
                    }
                    // sweep A over the j stored columns (lanes chosen for j).
                    const int nvr = j;
                    const int TA = nvr <= 8 ? 1 : (nvr <= 16 ? 2 : (nvr <= 32 ? 4 : 8));
                    const int PRA = WGS / TA;
                    const int sa = threadIdx.x & (TA - 1);
                    double c2r[JT], ccr[JT], acc[JT];
#pragma unroll
                    for (int q = 0; q < JT; ++q) {
                        const int k = sa + q * TA;
                        c2r[q] = k < nvr ? coef[k] : 0.0;
                        ccr[q] = k < nvr ? cc[k] : 0.0;
                        acc[q] = 0;
                    }
                    const double h2l = lag[0], ihn = lag[1];
                    double* vout = V + (int64_t)j * ld;
                    accn = 0;
                    double accd = 0;
                    for (int p0 = threadIdx.x / TA; p0 < np; p0 += U * PRA) {
                        double2 vv[U][JT], ww[U], yy[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int pp = p0 + u * PRA;
                            const bool ok = pp < np;
#pragma unroll
                            for (int q = 0; q < JT; ++q) {
                                const int k = sa + q * TA;
                                vv[u][q] = (ok && k < nvr) ? ld2(V + (int64_t)k * ld + 2 * pp) : make_double2(0.0, 0.0);
                            }
                            ww[u] = ok ? ld2(w + 2 * pp) : make_double2(0.0, 0.0);
                            yy[u] = ok ? ld2(y + 2 * pp) : make_double2(0.0, 0.0);
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int pp = p0 + u * PRA;
                            double a2x = 0, a2y = 0, a3x = 0, a3y = 0;
#pragma unroll
                            for (int q = 0; q < JT; ++q) {
                                a2x += vv[u][q].x * c2r[q];
                                a2y += vv[u][q].y * c2r[q];
                                a3x += vv[u][q].x * ccr[q];
                                a3y += vv[u][q].y * ccr[q];
                            }
                            a2x = gsum(a2x, TA);
                            a2y = gsum(a2y, TA);
                            a3x = gsum(a3x, TA);
                            a3y = gsum(a3y, TA);
                            if (pp >= np) continue;
                            const int i = 2 * pp;
                            double2 u2 = yy[u];
                            if (i + 1 >= n) u2.y = 0.0;
                            const double2 w2 = make_double2(ww[u].x - a2x, ww[u].y - a2y);
                            double2 wn = make_double2((u2.x - a3x - w2.x * h2l) * ihn,
                                                      (u2.y - a3y - w2.y * h2l) * ihn);
                            if (i + 1 >= n) wn.y = 0.0;
                            if (sa == 0) {
                                st2(vout + i, w2);
                                st2(w + i, wn);
                                accn += wn.x * wn.x + wn.y * wn.y;
                                accd += w2.x * wn.x + w2.y * wn.y;
                            }
#pragma unroll
                            for (int q = 0; q < JT; ++q) acc[q] += vv[u][q].x * wn.x + vv[u][q].y * wn.y;
                        }
                    }
                    bsum_cols<WGS, MB, JT>(acc, accn, nvr, TA, red, h1);
                    const double dj = bsum<WGS>(accd, sred);
                    wpre2 = h1[nvr];   // ||w||^2, the breakdown reference
                    __syncthreads();   // every wave has read it before the slot is reused
                    if (threadIdx.x == 0) h1[nvr] = dj;
                    __syncthreads();
                }
                for (int k = threadIdx.x; k < nv; k += WGS) {
                    h1[k] *= vscale[k];
                    coef[k] = h1[k] * vscale[k];
                }
                __syncthreads();
                // pass 2 (sweep B): w -= V coef; dots; ||w||^2
                double cr[JT], acc[JT];
#pragma unroll
                for (int q = 0; q < JT; ++q) {
                    const int k = sub + q * T;
                    cr[q] = k < nv ? coef[k] : 0.0;
                    acc[q] = 0;
                }
                accn = 0;
                for (int p0 = threadIdx.x / T; p0 < np; p0 += U * PR) {
                    double2 vv[U][JT], ww[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int pp = p0 + u * PR;
                        const bool ok = pp < np;
#pragma unroll
                        for (int q = 0; q < JT; ++q) {
                            const int k = sub + q * T;
                            vv[u][q] = (ok && k < nv) ? ld2(V + (int64_t)k * ld + 2 * pp) : make_double2(0.0, 0.0);
                        }
                        ww[u] = ok ? ld2(w + 2 * pp) : make_double2(0.0, 0.0);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int pp = p0 + u * PR;
                        double ux = 0, uy = 0;
#pragma unroll
                        for (int q = 0; q < JT; ++q) {
                            ux += vv[u][q].x * cr[q];
                            uy += vv[u][q].y * cr[q];
                        }
                        ux = gsum(ux, T);
                        uy = gsum(uy, T);
                        if (pp >= np) continue;
                        const double2 wv2 = make_double2(ww[u].x - ux, ww[u].y - uy);
                        if (sub == 0) {
                            st2(w + 2 * pp, wv2);
                            accn += wv2.x * wv2.x + wv2.y * wv2.y;
                        }
#pragma unroll
                        for (int q = 0; q < JT; ++q) acc[q] += vv[u][q].x * wv2.x + vv[u][q].y * wv2.y;
                    }
                }
                bsum_cols<WGS, MB, JT>(acc, accn, nv, T, red, h2);
                for (int k = threadIdx.x; k < nv; k += WGS) {
                    h2[k] *= vscale[k];
                    coef[k] = h2[k] * vscale[k];
                }
                __syncthreads();
                // Givens step of column j: H[:, j] = h1 + h2, h_{j+1,j} = hn with
                // hn^2 = ||w1||^2 - ||h2||^2 (the rounding of that difference is
                // about sqrt(eps) ||w|| -- the breakdown threshold).
                if (threadIdx.x == 0) {
                    double q2 = 0;
                    for (int i = 0; i <= j; ++i) q2 += h2[i] * h2[i];
                    const double hn = sqrt(fmax(h2[nv] - q2, 0.0));
                    const int bd = !(hn > 1.4901161193847656e-08 * sqrt(wpre2));
                    for (int i = 0; i <= j; ++i) Hr[i * MB + j] = h1[i] + h2[i];
                    Hr[(j + 1) * MB + j] = hn;
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
                    lag[0] = h2[j];
                    lag[1] = bd ? 0.0 : 1.0 / hn;
                    s_flag = (fabs(g[j + 1]) <= target || bd) ? 1 : 0;
                }
                __syncthreads();
                // Next step's c = H h2 on rows l <= j (band: columns l-1 .. j),
                // times vscale[l] (coefficients of the stored columns).
                for (int l = threadIdx.x; l <= j; l += WGS) {
                    double c = 0;
                    for (int k = (l > 0 ? l - 1 : 0); k <= j; ++k) c += Hr[l * MB + k] * h2[k];
                    cc[l] = c * vscale[l];
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
                for (int t = 0; t < kk; ++t) acc += V[(int64_t)t * ld + i] * coef[t];
                x[i] += acc;
            }
            __syncthreads();
        }
        // Final coarse correction x = x_hat + Z E^{-1} Z^T (b - A x_hat)
        // (svec holds E^{-1} Z^T r of the last restart).
        if (rho0 > 0.0 && R > 0) {
            for (int i = threadIdx.x; i < n; i += WGS) {
                double v = x[i];
                for (int q = a.zrp[r0 + i]; q < a.zrp[r0 + i + 1]; ++q) v += a.zv[q] * svec[a.zci[q] - c0];
                x[i] = v;
            }
        }
        // A system leaving for its continuation plan: each wave's x stores
        // reach memory (agent-scope release) before the flag below.
        if (status == kStatusHandoff && a.rec) __threadfence();
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
            if (status == kStatusHandoff && a.rec) {
                a.rec[sys].its = its;
                a.rec[sys].rho0 = rho0;
                __hip_atomic_store(&a.rec[sys].flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
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

GM_DEBUG_ACCESSOR(dbg_take_batched)

}  // namespace gm
