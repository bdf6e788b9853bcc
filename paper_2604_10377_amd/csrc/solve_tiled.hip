// Row systems of order 64 < k_x <= 319 (Eqs. (5)-(7) at large spectral
// resolution), and the adjoint products for any k.
//
// One 512-thread workgroup per row system (pair p, row i), persistent over the
// systems of the launch.  The lower triangle of S_i = K + lambda diag(D_i) is
// cut into 32x32 tiles, stored in LDS when they fit (k_x <= 223: 28 tiles) or
// in a per-workgroup slot of the workspace otherwise (L2 / last-level cache
// resident).  The right-hand side is appended as one extra row (index k_x), so
// the factorisation performs the forward substitution L y = r on the fly.
// Right-looking blocked Cholesky, step p:
//   1. wave 0 factorises the diagonal tile in registers (lane = row, column
//      broadcast through LDS) and forms L_pp^{-1} (one column per lane);
//   2. panel tiles: L_Ip = S_Ip L_pp^{-T}, a 32x32x32 product on the float32
//      matrix cores, one tile per wave;
//   3. trailing tiles: S_IJ -= L_Ip L_Jp^T on the matrix cores, one tile per
//      wave at a time.
// The back substitution L^T c = y then runs block column by block column.
// With stored factors (reverse mode) the tiles hold L and only the appended
// row is carried through steps 2-3.
#include "fmap_device.h"
#include "fmap_launch.h"

namespace fmap {

namespace {

constexpr int TLD = 33;                 // row stride of a stored tile (odd: conflict-free columns)
constexpr int TSZ = 32 * TLD;           // floats per tile
constexpr int LDD = 36;                 // row stride of the factorised diagonal tile (aligned rows)
constexpr int TW = 8;                   // waves per workgroup

__device__ __forceinline__ int packed_col_t(int c, int m) { return c * m - (c * (c - 1)) / 2; }
__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
// index of tile (I, J), I >= J, in column-major order of the lower triangle with TR tile rows
__device__ __forceinline__ int tile_index(int I, int J, int TR) { return J * TR - (J * (J - 1)) / 2 + (I - J); }

// LDS besides the tiles (floats)
constexpr int aux_floats(int TRM) { return TSZ /*minv*/ + 32 * LDD /*dl*/ + 32 /*bc*/ + 4 * TRM * 32 + 16; }

}  // namespace

enum { RT_FWD = 0, RT_BWD_STORED = 1, RT_BWD_RECOMPUTE = 2 };

// At TMAX = 4 the ten tiles take 40 KB of LDS: capped at 128 VGPRs (4 waves per SIMD, no spills),
// two workgroups, i.e. two systems, share a CU instead of one.
template <int TMAX, bool GT, int MODE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TMAX <= 4 ? 4 : 1))) void rowsolve_tiles_kernel(
    const float *__restrict__ K, const float *__restrict__ Lin, const float *__restrict__ rhs,
    const float *__restrict__ ex, const float *__restrict__ ey, const float *__restrict__ lam, int mask_kind,
    float gamma, int kx, int ky, int nsys, float *out, float *__restrict__ Lout, int *__restrict__ info,
    const float *__restrict__ Cfwd, float *__restrict__ dlam_part, float *__restrict__ tile_ws, const float *addend)
{
    constexpr int TRM = TMAX;                        // k_x + 1 rows fit in TMAX tile rows
    constexpr int NTL = TMAX * (TMAX + 1) / 2;
    constexpr bool STORED = MODE == RT_BWD_STORED;
    extern __shared__ __align__(16) float smem[];
    float *aux = GT ? smem : smem + NTL * TSZ;
    float *s_minv = aux;
    float *s_dl = s_minv + TSZ;
    float *s_bc = s_dl + 32 * LDD;
    float *s_vec = s_bc + 32;
    float *s_shift = s_vec + TRM * 32;
    float *s_dval = s_shift + TRM * 32;
    float *s_part = s_dval + TRM * 32;
    float *s_red = s_part + TRM * 32;
    int *s_fail = reinterpret_cast<int *>(s_red + 8);
    float *tiles = GT ? tile_ws + (size_t)blockIdx.x * NTL * TSZ : smem;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, half = lane >> 5;
    const int T = (kx + 31) >> 5;   // column tiles
    const int TR = (kx + 32) >> 5;  // tile rows (row kx is the right-hand side)
    const int AR = kx >> 5, ar = kx & 31;

    for (int sys = blockIdx.x; sys < nsys; sys += gridDim.x) {
        const int p = sys / ky, i = sys % ky;
        // ---- lambda, mask row, normaliser ---------------------------------------------
        const float lamv = lam[p];
        int fail0 = (!(lamv >= 0.f) || !isfinite(lamv)) ? -1 : 0;
        MaskParams mp;
        mp.kind = mask_kind;
        mp.gamma = gamma;
        mp.inv_scale = 1.f;
        if (mask_kind == 1) {
            float mx = -INFINITY;
            for (int q = tid; q < kx; q += 512) mx = fmaxf(mx, ex[(size_t)p * kx + q]);
            for (int q = tid; q < ky; q += 512) mx = fmaxf(mx, ey[(size_t)p * ky + q]);
            mx = wave_max(mx);
            if (lane == 0) s_red[wave] = mx;
            __syncthreads();
            mx = s_red[0];
#pragma unroll
            for (int w = 1; w < TW; ++w) mx = fmaxf(mx, s_red[w]);
            if ((!(mx > 0.f) || !isfinite(mx)) && fail0 == 0) fail0 = -2;
            mp.inv_scale = 1.f / mx;
        }
        const float muy = ey[(size_t)p * ky + i];
        for (int q = tid; q < TRM * 32; q += 512) {
            const float dv = (q < kx && fail0 != -2) ? mask_entry(muy, ex[(size_t)p * kx + q], mp) : 0.f;
            s_dval[q] = dv;
            s_shift[q] = fail0 == 0 ? lamv * dv : 0.f;
            s_vec[q] = 0.f;
        }
        if (tid == 0) *s_fail = fail0;
        __syncthreads();

        // ---- tiles: S (lower, shifted diagonal) or L; appended row = right-hand side ----
        const float *Kp = STORED ? nullptr : K + (size_t)p * kx * kx;
        const float *Lp = STORED ? Lin + ((size_t)p * ky + i) * (size_t)(kx * (kx + 1) / 2) : nullptr;
        const float *rp = rhs + ((size_t)p * ky + i) * kx;
        // tiles in column-major order of the lower triangle, two entries per thread per tile, TG tiles
        // at a time: their loads are unconditional (addresses clamped into the arrays, the right-hand
        // side row selected by address) so all of a group's loads are in flight together, and the
        // values are masked when written
        {
            constexpr int TG = 4;
            const int ntile = T * TR - (T * (T - 1)) / 2;
            int I = 0, J = 0;  // tile cursor, uniform
            for (int tau0 = 0; tau0 < ntile; tau0 += TG) {
                float v[TG][2];
                int Iu[TG], Ju[TG];
#pragma unroll
                for (int u = 0; u < TG; ++u) {
                    Iu[u] = I;
                    Ju[u] = J;
                    if (++I >= TR) {  // next column of tiles
                        ++J;
                        I = J;
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int rc = tid + 512 * h, r = rc >> 5, c = rc & 31;
                        const int row = min(32 * Iu[u] + r, kx), col = min(32 * Ju[u] + c, kx - 1);
                        const float *src;
                        if (STORED) {
                            const int cc = min(col, min(row, kx - 1));
                            src = row == kx ? rp + col : Lp + packed_col_t(cc, kx) + min(row, kx - 1) - cc;
                        } else {
                            src = row == kx ? rp + col : Kp + (size_t)row * kx + col;
                        }
                        v[u][h] = *src;
                    }
                }
#pragma unroll
                for (int u = 0; u < TG; ++u) {
                    if (tau0 + u >= ntile) break;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int rc = tid + 512 * h, r = rc >> 5, c = rc & 31;
                        const int row = 32 * Iu[u] + r, col = 32 * Ju[u] + c;
                        float x = 0.f;
                        if (row < kx && col <= row) x = STORED ? v[u][h] : v[u][h] + (row == col ? s_shift[row] : 0.f);
                        else if (row == kx && col < kx) x = v[u][h];
                        tiles[(tau0 + u) * TSZ + r * TLD + c] = x;
                    }
                }
            }
        }
        __syncthreads();

        for (int pstep = 0; pstep < T; ++pstep) {
            if (__builtin_amdgcn_readfirstlane(*s_fail) != 0) break;
            const int kxl = min(32, kx - 32 * pstep);
            float *Dt = tiles + tile_index(pstep, pstep, TR) * TSZ;
            // 1. diagonal tile and L_pp^{-1} (wave 0)
            if (wave == 0) {
                float sr[32];
#pragma unroll
                for (int q = 0; q < 32; ++q) sr[q] = (lane < 32) ? Dt[l32 * TLD + q] : 0.f;
                int fail = 0;
                // column c of L: the pivot and the entries L_qc come from the lanes that hold rows c and q
                // (readlane, no LDS round trip); lane j updates its row; entries above the diagonal are
                // updated too but never read again
#pragma unroll
                for (int c = 0; c < 32; ++c) {
                    if (c < kxl && fail == 0) {
                        const float piv = uniform_f(readlane(sr[c], c));
                        if (!(piv > 0.f) || !isfinite(piv)) {
                            fail = 32 * pstep + c + 1;
                        } else if (!STORED) {
                            const float l = sr[c] * __builtin_amdgcn_rsqf(piv);
                            sr[c] = l;
#pragma unroll
                            for (int q = c + 1; q < 32; ++q) sr[q] -= l * readlane(l, q);
                        }
                    }
                }
                if (fail == 0 && lane < 32 && !STORED) {
#pragma unroll
                    for (int q = 0; q < 32; ++q) Dt[l32 * TLD + q] = sr[q];
                }
                if (lane == 0 && fail != 0) *s_fail = fail;
                if (fail == 0) {
                    // column `lane` of L_pp^{-1}: m_q = (delta_{q,lane} - sum_{t<q} L_qt m_t) / L_qq, the
                    // entries of L read from the lanes holding them
                    float m[32];
#pragma unroll
                    for (int q = 0; q < 32; ++q) {
                        float t = (q == lane) ? 1.f : 0.f;
#pragma unroll
                        for (int tt = 0; tt < q; ++tt) t -= readlane(sr[tt], q) * m[tt];
                        m[q] = (q < kxl) ? t * __builtin_amdgcn_rcpf(readlane(sr[q], q)) : 0.f;
                    }
                    if (lane < 32) {
#pragma unroll
                        for (int q = 0; q < 32; ++q) s_minv[q * TLD + l32] = m[q];  // Minv[q][lane]
                    }
                }
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(*s_fail) != 0) break;

            // 2. panel tiles (I, pstep), I > pstep: L_Ip = S_Ip Minv^T
            {
                const int first = pstep + 1;
                const int npan = STORED ? (AR > pstep ? 1 : 0) : TR - first;
                for (int q = wave; q < npan; q += TW) {
                    const int I = STORED ? AR : first + q;
                    float *X = tiles + tile_index(I, pstep, TR) * TSZ;
                    f32x16 nv = zero16();
#pragma unroll
                    for (int t = 0; t < 16; ++t)
                        nv = mfma32x32x2(X[l32 * TLD + 2 * t + half], s_minv[l32 * TLD + 2 * t + half], nv);
                    __builtin_amdgcn_wave_barrier();
                    // with stored factors the tile's other rows are final L rows: only the appended row moves
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (!STORED || acc32_row(r, lane) == ar) X[acc32_row(r, lane) * TLD + l32] = nv[r];
                }
                if (STORED && AR == pstep && wave == 0) {
                    // appended row inside the diagonal tile: y_c = sum_t Minv[c][t] s_t
                    float y = 0.f;
                    if (lane < kxl) {
#pragma unroll
                        for (int t = 0; t < 32; ++t) y += s_minv[l32 * TLD + t] * Dt[ar * TLD + t];
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (lane < 32) Dt[ar * TLD + l32] = (lane < kxl) ? y : 0.f;
                }
            }
            __syncthreads();

            // 3. trailing tiles (I, J), pstep < J <= I < TR: S_IJ -= L_Ip L_Jp^T
            {
                const int nt = TR - pstep - 1;  // block columns pstep+1 .. TR-1 of the trailing part
                const int ntrail = STORED ? (AR > pstep ? AR - pstep : 0) : nt * (nt + 1) / 2;
                for (int q = wave; q < ntrail; q += TW) {
                    int I, J;
                    if (STORED) {
                        I = AR;
                        J = pstep + 1 + q;
                    } else {
                        int jj = 0, t2 = q;
                        while (t2 >= nt - jj) {
                            t2 -= nt - jj;
                            ++jj;
                        }
                        J = pstep + 1 + jj;
                        I = J + t2;
                    }
                    if (J >= T) continue;  // the appended row's block beyond the last column
                    float *X = tiles + tile_index(I, J, TR) * TSZ;
                    const float *LI = tiles + tile_index(I, pstep, TR) * TSZ;
                    const float *LJ = tiles + tile_index(J, pstep, TR) * TSZ;
                    f32x16 acc;
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[r] = X[acc32_row(r, lane) * TLD + l32];
#pragma unroll
                    for (int t = 0; t < 16; ++t)
                        acc = mfma32x32x2(-LI[l32 * TLD + 2 * t + half], LJ[l32 * TLD + 2 * t + half], acc);
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (!STORED || acc32_row(r, lane) == ar) X[acc32_row(r, lane) * TLD + l32] = acc[r];
                }
            }
            // y of this block column (the appended row) is final
            if (wave == TW - 1 && lane < 32) {
                const float *src = tiles + tile_index(AR, pstep, TR) * TSZ;
                s_vec[32 * pstep + l32] = (l32 < kxl) ? src[ar * TLD + l32] : 0.f;
            }
            __syncthreads();
        }
        const int fail = __builtin_amdgcn_readfirstlane(*s_fail);

        // ---- factors out (forward mode) ----------------------------------------------------
        if (MODE == RT_FWD && Lout && fail == 0) {
            // in packed (column-major) order, so consecutive threads store consecutive floats.  Entry e
            // lies in the column q with packed_col(q) <= e < packed_col(q + 1), found from the quadratic
            // for packed_col (hardware square root) and corrected by one step either way; every index
            // product fits in 24 bits
            float *Lo = Lout + ((size_t)p * ky + i) * (size_t)(kx * (kx + 1) / 2);
            const int total = kx * (kx + 1) / 2;
            const unsigned ku = (unsigned)kx;
            auto pcol = [&](unsigned q) { return __umul24(q, ku) - (__umul24(q, q - 1u) >> 1); };
            const float bq = 2.f * kx + 1.f;
            // 8 entries per batch: their LDS reads are issued together, then the stores
            for (int e0 = tid; e0 < total; e0 += 8 * 512) {
                int src[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const unsigned e = (unsigned)min(e0 + 512 * u, total - 1);
                    unsigned q = (unsigned)max(
                        (int)((bq - __builtin_amdgcn_sqrtf(fmaxf(bq * bq - 8.f * (float)e, 0.f))) * 0.5f), 0);
                    q = min(q, ku - 1u);
                    q += (unsigned)((q + 1u < ku) & (pcol(q + 1u) <= e));
                    q -= (unsigned)((q > 0u) & (pcol(q) > e));
                    const int col = (int)q, row = (int)min(q + e - pcol(q), ku - 1u);
                    src[u] = tile_index(row >> 5, col >> 5, TR) * TSZ + (row & 31) * TLD + (col & 31);
                }
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = tiles[src[u]];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (e0 + 512 * u < total) Lo[e0 + 512 * u] = v[u];
            }
        }

        // ---- back substitution L^T c = y ----------------------------------------------------
        if (fail == 0) {
            for (int pstep = T - 1; pstep >= 0; --pstep) {
                const int kxl = min(32, kx - 32 * pstep);
                // z_I = L_Ip^T c_I for pstep < I < T: lanes 0..31 and 32..63 take two tiles
                const int nz = T - pstep - 1;
                for (int q = 2 * wave + half; q < nz; q += 2 * TW) {
                    const int I = pstep + 1 + q;
                    const float *X = tiles + tile_index(I, pstep, TR) * TSZ;
                    float z = 0.f;
#pragma unroll
                    for (int r = 0; r < 32; ++r) z += X[r * TLD + l32] * s_vec[32 * I + r];
                    s_part[32 * I + l32] = z;
                }
                __syncthreads();
                if (wave == 0) {
                    const float *Dt = tiles + tile_index(pstep, pstep, TR) * TSZ;
                    float v = 0.f;
                    if (lane < 32) {
                        v = s_vec[32 * pstep + l32];
                        for (int I = pstep + 1; I < T; ++I) v -= s_part[32 * I + l32];
                    }
                    float cv = 0.f;
#pragma unroll
                    for (int c = 31; c >= 0; --c) {
                        if (c < kxl) {
                            const float cc = readlane(v, c) * __builtin_amdgcn_rcpf(Dt[c * TLD + c]);
                            if (lane == c) cv = cc;
                            if (lane < c) v -= Dt[c * TLD + l32] * cc;
                        }
                    }
                    if (lane < 32) s_vec[32 * pstep + l32] = (l32 < kxl) ? cv : 0.f;
                }
                __syncthreads();
            }
        }

        // ---- outputs ----------------------------------------------------------------------
        for (int q = tid; q < kx; q += 512) {
            const size_t o = ((size_t)p * ky + i) * kx + q;
            const float v = fail == 0 ? s_vec[q] : NAN;
            out[o] = addend ? addend[o] + v : v;  // addend: refinement correction c += delta (in place)
        }
        if (info && tid == 0) info[(size_t)p * ky + i] = fail;
        if (MODE != RT_FWD && dlam_part) {
            float term = 0.f;
            for (int q = tid; q < kx; q += 512)
                term += (fail == 0 ? s_vec[q] : NAN) * s_dval[q] * Cfwd[((size_t)p * ky + i) * kx + q];
            term = wave_sum(term);
            if (lane == 0) s_red[wave] = term;
            __syncthreads();
            if (tid == 0) {
                float sm = 0.f;
#pragma unroll
                for (int w = 0; w < TW; ++w) sm += s_red[w];
                dlam_part[(size_t)p * ky + i] = -sm;
            }
        }
        __syncthreads();  // LDS and the tile slot are reused by the next system
    }
}

// ---------------------------------------------------------------------------
// Batched products for the adjoint at any k (operands streamed from global
// memory / L2).  Out[p] (M x N, row-major) = sum over two K-segments s of
// sign_s * X_s Y_s, where X_s is M x K_s read as stored ("N") or as the
// transpose of a K_s x M row-major array ("T"), and Y_s is K_s x N row-major.
// One wave per 32x32 output tile; loads are issued in batches of 8 steps.
// ---------------------------------------------------------------------------
struct GemmSeg {
    const float *X;
    const float *Y;
    int K;
    int transX;  // 1: X given as K x M row-major
    int ldx, ldy;
    long long strideX, strideY;  // per pair
    float sign;
};

__global__ __launch_bounds__(256) void batched_gemm_kernel(GemmSeg s0, GemmSeg s1, int nseg, int M, int N,
                                                           int tilesM, int tilesN, long long nwaves,
                                                           float *__restrict__ Out, long long strideO)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int tiles = tilesM * tilesN;
    const long long gtile = (long long)blockIdx.x * 4 + wave;
    if (gtile >= nwaves) return;
    const int p = (int)(gtile / tiles);
    const int t = (int)(gtile % tiles);
    const int I = t / tilesN, Jt = t % tilesN;
    const int m = I * 32 + l32, n = Jt * 32 + l32;
    const bool mok = m < M, nok = n < N;
    f32x16 acc = zero16();
    for (int sgi = 0; sgi < nseg; ++sgi) {
        const GemmSeg &sg = sgi == 0 ? s0 : s1;
        const float *X = sg.X + (long long)p * sg.strideX;
        const float *Y = sg.Y + (long long)p * sg.strideY;
        // every load unconditional, from addresses clamped into the operands, and masked by a bit mask
        // afterwards: a load under a condition was compiled as a branch with a wait of its own, and the
        // batch's loads then went out one at a time
        const int mc = min(m, M - 1), nc = min(n, N - 1);
        auto keep = [](float x, bool ok) { return __uint_as_float(__float_as_uint(x) & (ok ? ~0u : 0u)); };
        for (int k0 = 0; k0 < sg.K; k0 += 16) {
            float a[8], b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = k0 + 2 * u + half;
                const int kc = min(kk, sg.K - 1);
                const size_t xo = sg.transX ? (size_t)kc * sg.ldx + mc : (size_t)mc * sg.ldx + kc;
                a[u] = X[xo];
                b[u] = Y[(size_t)kc * sg.ldy + nc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool kok = k0 + 2 * u + half < sg.K;
                a[u] = keep(sg.sign * a[u], mok && kok);
                b[u] = keep(b[u], nok && kok);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = mfma32x32x2(a[u], b[u], acc);
        }
    }
    float *O = Out + (long long)p * strideO;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = I * 32 + acc32_row(r, lane);
        if (row < M && nok) O[(size_t)row * N + n] = acc[r];
    }
}

// Sum of the per-row dlambda terms of each pair, in row order.
__global__ void dlam_sum_kernel(const float *__restrict__ part, int P, int ky, float *__restrict__ dlam)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = 0.f;
    for (int i = 0; i < ky; ++i) s += part[(size_t)p * ky + i];
    dlam[p] = s;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static int cu_count()
{
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) return 256;
    return c;
}

// Workgroups of a launch whose tiles live in the workspace (one tile slot each).
static int64_t tiled_global_slots(int64_t nsys)
{
    const int64_t cap = 2 * (int64_t)cu_count();
    return nsys < cap ? nsys : cap;
}

size_t tiled_workspace_bytes(int64_t P, int64_t kx, int64_t ky)
{
    if (kx < 224) return 0;
    const int64_t ntl = 10 * 11 / 2;
    return (size_t)tiled_global_slots(P * ky) * ntl * TSZ * sizeof(float);
}

template <int TMAX, bool GT, int MODE>
static void launch_tiles(const float *K, const float *Lin, const float *rhs, const float *ex, const float *ey,
                         const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky, float *out,
                         float *Lout, int *info, const float *Cfwd, float *dlam_part, float *tws, hipStream_t st,
                         const float *addend)
{
    constexpr int NTL = TMAX * (TMAX + 1) / 2;
    const size_t lds = ((GT ? 0 : (size_t)NTL * TSZ) + aux_floats(TMAX)) * sizeof(float);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)rowsolve_tiles_kernel<TMAX, GT, MODE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    const int64_t nsys = P * ky;
    const int64_t grid = GT ? tiled_global_slots(nsys) : nsys;
    hipLaunchKernelGGL((rowsolve_tiles_kernel<TMAX, GT, MODE>), dim3((unsigned)grid), dim3(512), lds, st, K, Lin, rhs,
                       ex, ey, lam, mask_kind, gamma, (int)kx, (int)ky, (int)nsys, out, Lout, info, Cfwd, dlam_part,
                       tws, addend);
}

template <int MODE>
static void launch_tiled_mode(const float *K, const float *Lin, const float *rhs, const float *ex, const float *ey,
                              const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx, int64_t ky,
                              float *out, float *Lout, int *info, const float *Cfwd, float *dlam_part, float *tws,
                              hipStream_t st, const float *addend)
{
    if (kx < 128)
        launch_tiles<4, false, MODE>(K, Lin, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info, Cfwd,
                                     dlam_part, tws, st, addend);
    else if (kx < 224)
        launch_tiles<7, false, MODE>(K, Lin, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info, Cfwd,
                                     dlam_part, tws, st, addend);
    else
        launch_tiles<10, true, MODE>(K, Lin, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info, Cfwd,
                                     dlam_part, tws, st, addend);
}

void launch_rowsolve_tiled(int mode, const float *K, const float *Lin, const float *rhs, const float *ex,
                           const float *ey, const float *lam, int mask_kind, float gamma, int64_t P, int64_t kx,
                           int64_t ky, float *out, float *Lout, int *info, const float *Cfwd, float *dlam_part,
                           float *tws, hipStream_t st, const float *addend)
{
    if (mode == RT_FWD)
        launch_tiled_mode<RT_FWD>(K, Lin, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info, Cfwd,
                                  dlam_part, tws, st, addend);
    else if (mode == RT_BWD_STORED)
        launch_tiled_mode<RT_BWD_STORED>(K, Lin, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info, Cfwd,
                                         dlam_part, tws, st, addend);
    else
        launch_tiled_mode<RT_BWD_RECOMPUTE>(K, Lin, rhs, ex, ey, lam, mask_kind, gamma, P, kx, ky, out, Lout, info,
                                            Cfwd, dlam_part, tws, st, addend);
}

static void gemm(const GemmSeg &s0, const GemmSeg *s1, int64_t P, int M, int N, float *Out, long long strideO,
                 hipStream_t st)
{
    const int tM = (M + 31) / 32, tN = (N + 31) / 32;
    const long long waves = (long long)P * tM * tN;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    GemmSeg z = s0;
    z.K = 0;
    hipLaunchKernelGGL(batched_gemm_kernel, dim3(grid), dim3(256), 0, st, s0, s1 ? *s1 : z, s1 ? 2 : 1, M, N, tM, tN,
                       waves, Out, strideO);
}

// W = V^T C + C^T V (into Wbuf), dB = V A, dA = V^T B - W A.
void launch_adjoint_general(const float *V, const float *C, const float *A, const float *B, int64_t P, int64_t kx,
                            int64_t ky, int64_t d, float *Wbuf, const float *dlam_part, float *dlam, float *dA,
                            float *dB, hipStream_t st)
{
    const long long skk = kx * ky, sxd = kx * d, syd = ky * d, sww = kx * kx;
    GemmSeg w0{V, C, (int)ky, 1, (int)kx, (int)kx, skk, skk, 1.f};
    GemmSeg w1{C, V, (int)ky, 1, (int)kx, (int)kx, skk, skk, 1.f};
    gemm(w0, &w1, P, (int)kx, (int)kx, Wbuf, sww, st);
    GemmSeg b0{V, A, (int)kx, 0, (int)kx, (int)d, skk, sxd, 1.f};
    gemm(b0, nullptr, P, (int)ky, (int)d, dB, syd, st);
    GemmSeg a0{V, B, (int)ky, 1, (int)kx, (int)d, skk, syd, 1.f};
    GemmSeg a1{Wbuf, A, (int)kx, 1, (int)kx, (int)d, sww, sxd, -1.f};  // W symmetric: W^T = W
    gemm(a0, &a1, P, (int)kx, (int)d, dA, sxd, st);
    if (dlam)
        hipLaunchKernelGGL(dlam_sum_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, dlam_part, (int)P,
                           (int)ky, dlam);
}

}  // namespace fmap
