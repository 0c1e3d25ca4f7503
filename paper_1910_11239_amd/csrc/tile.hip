// Local solves of 3-D vertex patches with 16-bit contractions, every 1-D
// contraction on MFMA and the overlapping patches summed by the workgroup that
// owns their cells (the FTS_SCHEDULE_OWNER schedule of fts_schwarz_apply).
#include <algorithm>

#include "device_common.h"

namespace fts {

typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// 16-bit local solves of 3-D vertex patches with every contraction on MFMA
// and the overlapping patches summed by their owners (no staging buffer).
//
// One wave holds one patch tensor T[z][y][x] (padded to 16^3) in registers:
// lane (q, j) = (l / 16, l % 16) keeps x = 4q..4q+3 of line y = j for all 16
// z.  With D = A B on v_mfma_f32_16x16x16 (lane (q, j) supplies A[j][4q+v]
// and B[4q+v][j] and receives D[4q+v][j]) the six contractions chain as
//   x fwd:  U_z = T_z F_x^T          (T_z as A, rows y)       -> U[y][m0]
//   y fwd:  V_z = F_y U_z            (U_z as B)                -> V[m1][m0]
//   z <-> m1 exchange across the four lane groups (permlane swaps)
//   z fwd:  W_m1 = F_z V_m1 ; scale ; z bwd: X_m1 = B_z W_m1   (as B)
//   m1 <-> z exchange back
//   y bwd:  Y_z = X_z^T B_y^T        (X_z^T as A, rows m0)     -> Y[m0][y]
//   x bwd:  C_z = B_x Y_z            (Y_z as B)                -> C[x][y]
// so the correction leaves in the layout the residual came in, and every
// operand is the previous result rounded to 16 bits.  F = S^T / s and
// B = S / s are the range-normalised tables of the other MFMA kernel, the
// residual is divided by its max-norm and the scaling uses
// Lambda_min / Lambda(m); the factor |r|_max omega (s_x s_y s_z)^2 /
// Lambda_min is applied when the correction is accumulated (FP32).
//
// Ownership: a workgroup owns a tile of TT x TT cells in x and y and a
// segment of cell layers along z, and computes every patch that touches its
// cells (patches on the tile border are computed by each neighbouring tile,
// which keeps only its own cells).  It marches along z through the vertex
// planes: the patches of one plane go in four rounds by the parity of their
// vertex in x and y (patches of one round share no cell), one patch per wave,
// and add their corrections into FP32 accumulators in LDS for the two cell
// layers the plane touches.  After a plane the lower layer has all its
// contributions; x is updated there once and its accumulator reused.
// Summation order is fixed, so results are deterministic.
constexpr int kTile = 3;

struct TileGrid {
    int nt[2];     // tiles along x and y
    int nseg;      // segments along z
    int zlen;      // cell layers per segment
    int ntile;     // nt[0] * nt[1] * nseg
    int per_xcd;   // tiles per XCD slot (block b -> tile (b % 8) * per_xcd + b / 8)
};

__device__ __forceinline__ unsigned pk16(float a, float b, int bf) {
    if (bf) {
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = {a, b};
        return __builtin_bit_cast(unsigned, __builtin_convertvector(v, b2));
    } else {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = {a, b};
        return __builtin_bit_cast(unsigned, __builtin_convertvector(v, h2));
    }
}

template <int BF>
__device__ __forceinline__ f32x4 mma_u(unsigned a0, unsigned a1, unsigned b0, unsigned b1) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 a = {a0, a1}, b = {b0, b1};
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    if constexpr (BF) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b),
                                                         z, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b), z,
                                                     0, 0, 0);
    }
}

// Exchange of a 4 x 4 block structure between the lane groups q = l / 16 and
// the register index h of P[h] (P[h][p] for p < NP): afterwards lane group q
// register h holds what lane group h register q held.  permlane32_swap swaps
// the upper half of the first operand with the lower half of the second
// (bit 1 of q with bit 1 of h), permlane16_swap the odd 16-lane rows of the
// first with the even rows of the second (bit 0).
template <int NP>
__device__ __forceinline__ void lanegroup_transpose(unsigned (&P)[4][NP]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const auto s = __builtin_amdgcn_permlane32_swap(P[h][p], P[h + 2][p], false, false);
            P[h][p] = s[0];
            P[h + 2][p] = s[1];
        }
#pragma unroll
    for (int h = 0; h < 4; h += 2)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const auto s = __builtin_amdgcn_permlane16_swap(P[h][p], P[h + 1][p], false, false);
            P[h][p] = s[0];
            P[h + 1][p] = s[1];
        }
}

template <int N1, int BF, typename TR>
__global__ void __launch_bounds__(256)
k_schwarz_mfma_tile(LevelView g, EigView e, TileGrid tg, const TR *__restrict__ r, double *__restrict__ x,
                    float omega) {
    constexpr int N = 2 * N1, NC1 = N1 * N1 * N1;
    static_assert(N <= 16, "one 16 x 16 tile per contraction");
    constexpr int CP = NC1 + 4;  // accumulator pitch per cell (offsets the banks of neighbouring cells)
    __shared__ float acc[2 * kTile * kTile * CP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int q = lane >> 4, j = lane & 15;
    const int b = blockIdx.x;
    const int tile = (b & 7) * tg.per_xcd + (b >> 3);
    if (tile >= tg.ntile) return;  // uniform per workgroup, before any barrier
    const int seg = tile / (tg.nt[0] * tg.nt[1]);
    const int txy = tile % (tg.nt[0] * tg.nt[1]);
    const int cx0 = kTile * (txy % tg.nt[0]), cy0 = kTile * (txy / tg.nt[0]);
    const int m0 = g.m[0], m1 = g.m[1], m2 = g.m[2];
    const int z0 = seg * tg.zlen, z1 = min(m2, z0 + tg.zlen);
    const int64_t cs1 = m0, cs2 = (int64_t)m0 * m1;
    for (int p = t; p < 2 * kTile * kTile * CP; p += 256) acc[p] = 0.f;
    __syncthreads();

    // flush cell layer L of the tile: x += acc, then clear the accumulator
    auto flush = [&](int L) {
        const int bufo = (L & 1) * kTile * kTile * CP;
        for (int e2 = t; e2 < kTile * kTile * NC1; e2 += 256) {
            const int c = e2 / NC1, o = e2 % NC1;
            const int cx = cx0 + c % kTile, cy = cy0 + c / kTile;
            if (cx < m0 && cy < m1) {
                double *xp = x + ((int64_t)L * cs2 + (int64_t)cy * cs1 + cx) * NC1 + o;
                *xp += (double)acc[bufo + c * CP + o];
            }
            acc[bufo + c * CP + o] = 0.f;
        }
    };

    const int vz_lo = max(z0, 1), vz_hi = min(z1, m2 - 1);
    for (int vz = vz_lo; vz <= vz_hi; ++vz) {
        for (int round = 0; round < 4; ++round) {
            const int px = round & 1, py = round >> 1;
            const int vx = cx0 + ((px - cx0) & 1) + 2 * (w & 1);
            const int vy = cy0 + ((py - cy0) & 1) + 2 * (w >> 1);
            const bool valid = vx >= 1 && vx <= m0 - 1 && vy >= 1 && vy <= m1 - 1 && vx <= cx0 + kTile &&
                               vy <= cy0 + kTile;
            if (valid) {  // uniform per wave
                const int pos[3] = {vx - 1, vy - 1, vz - 1};
                int tp[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) tp[a] = __builtin_amdgcn_readfirstlane(e.cls[a][pos[a]]);
                const int64_t cbase = pos[0] + pos[1] * cs1 + pos[2] * cs2;
                // residual of the patch: lane (q, j) reads x = 4q..4q+3 of line y = j, all z
                float rv[16][4];
                float amax = 0.f;
#pragma unroll
                for (int s = 0; s < 16; ++s) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) rv[s][i] = 0.f;
                    if (s < N && j < N) {
                        const int oz = s / N1, iz = s % N1, oy = j / N1, iy = j % N1;
                        if constexpr (N1 % 4 == 0) {
                            if (4 * q < N) {
                                const int ox = (4 * q) / N1, ix = (4 * q) % N1;
                                const TR *src = r + (cbase + ox + oy * cs1 + oz * cs2) * NC1 + iz * N1 * N1 +
                                                iy * N1 + ix;
                                if constexpr (sizeof(TR) == 8) {
                                    const double2 u0 = *reinterpret_cast<const double2 *>(src);
                                    const double2 u1 = *reinterpret_cast<const double2 *>(src + 2);
                                    rv[s][0] = (float)u0.x;
                                    rv[s][1] = (float)u0.y;
                                    rv[s][2] = (float)u1.x;
                                    rv[s][3] = (float)u1.y;
                                } else {
                                    const float4 u = *reinterpret_cast<const float4 *>(src);
                                    rv[s][0] = u.x;
                                    rv[s][1] = u.y;
                                    rv[s][2] = u.z;
                                    rv[s][3] = u.w;
                                }
                            }
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const int a0 = 4 * q + i;
                                if (a0 < N) {
                                    const int ox = a0 / N1, ix = a0 % N1;
                                    rv[s][i] = (float)r[(cbase + ox + oy * cs1 + oz * cs2) * NC1 + iz * N1 * N1 +
                                                        iy * N1 + ix];
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) amax = fmaxf(amax, fabsf(rv[s][i]));
                }
                for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
                const float inv = amax > 0.f ? 1.f / amax : 0.f;
                auto tab = [&](const uint16_t *const *tb, int a, unsigned &u0, unsigned &u1) {
                    const uint2 u = *reinterpret_cast<const uint2 *>(tb[a] + (size_t)tp[a] * 256 + j * 16 + 4 * q);
                    u0 = u.x;
                    u1 = u.y;
                };
                const uint16_t *const *Ft = BF ? e.Fbf16 : e.Ff16;
                const uint16_t *const *Bt = BF ? e.Bbf16 : e.Bf16;
                unsigned fx0, fx1, fy0, fy1, fz0, fz1, bz0, bz1, by0, by1, bx0, bx1;
                tab(Ft, 0, fx0, fx1);
                tab(Ft, 1, fy0, fy1);
                tab(Ft, 2, fz0, fz1);
                tab(Bt, 2, bz0, bz1);
                tab(Bt, 1, by0, by1);
                tab(Bt, 0, bx0, bx1);
                // forward x and y per z slice; V packed for the exchange:
                // P[h][2 sp + i / 2]... indexed P[h][sp * 4 + i] = (V[4h+2sp][i], V[4h+2sp+1][i])
                unsigned P[4][8];
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int sp = 0; sp < 2; ++sp) {
                        f32x4 Vp[2];
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const int s = 4 * h + 2 * sp + u;
                            const unsigned a0 = pk16(rv[s][0] * inv, rv[s][1] * inv, BF);
                            const unsigned a1 = pk16(rv[s][2] * inv, rv[s][3] * inv, BF);
                            const f32x4 U = mma_u<BF>(a0, a1, fx0, fx1);
                            Vp[u] = mma_u<BF>(fy0, fy1, pk16(U[0], U[1], BF), pk16(U[2], U[3], BF));
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) P[h][sp * 4 + i] = pk16(Vp[0][i], Vp[1][i], BF);
                    }
                lanegroup_transpose<8>(P);
                // now P[h][sp * 4 + i] holds V[z = 4q + 2sp + {0,1}][m1 = 4h + i][m0 = j]
                const float *lx = e.lam32[0] + (size_t)tp[0] * N, *ly = e.lam32[1] + (size_t)tp[1] * N;
                const float *lz = e.lam32[2] + (size_t)tp[2] * N;
                const float lmin = e.lmin[0][tp[0]] + e.lmin[1][tp[1]] + e.lmin[2][tp[2]];
                // Lambda(m) / Lambda_min = axz[v] + ly[m1] / Lambda_min; its
                // reciprocal by v_rcp_f32 (about 1 ulp, far below the 16-bit rounding)
                const float ilmin = 1.f / lmin;
                const float lxj = j < N ? lx[j] : 0.f;
                float axz[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) axz[i] = (4 * q + i < N) ? (lxj + lz[4 * q + i]) * ilmin : 0.f;
                unsigned Q[4][8];
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int pp = 0; pp < 2; ++pp) {
                        f32x4 Xp[2];
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const int m1i = 4 * h + 2 * pp + u, i = m1i & 3;
                            f32x4 W = mma_u<BF>(fz0, fz1, P[h][i], P[h][4 + i]);
                            const float lyv = (m1i < N) ? ly[m1i] * ilmin : 0.f;
                            const bool inxy = j < N && m1i < N;
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                W[v] = (inxy && 4 * q + v < N) ? W[v] * __builtin_amdgcn_rcpf(axz[v] + lyv) : 0.f;
                            Xp[u] = mma_u<BF>(bz0, bz1, pk16(W[0], W[1], BF), pk16(W[2], W[3], BF));
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) Q[h][pp * 4 + v] = pk16(Xp[0][v], Xp[1][v], BF);
                    }
                lanegroup_transpose<8>(Q);
                // now Q[h][pp * 4 + v] holds X[m1 = 4q + 2pp + {0,1}][z = 4h + v][m0 = j]
                const double sx = e.mscale[0][tp[0]], sy = e.mscale[1][tp[1]], sz = e.mscale[2][tp[2]];
                const float Fs = (float)((double)amax * (double)omega * (sx * sy * sz) * (sx * sy * sz) /
                                         (double)lmin);
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int zz = 4 * h + v;
                        const f32x4 Y = mma_u<BF>(Q[h][v], Q[h][4 + v], by0, by1);
                        const f32x4 C = mma_u<BF>(bx0, bx1, pk16(Y[0], Y[1], BF), pk16(Y[2], Y[3], BF));
                        // C[x = 4q + i][y = j] of slice z = zz
                        if (zz < N && j < N) {
                            const int oz = zz / N1, iz = zz % N1, oy = j / N1, iy = j % N1;
                            const int L = pos[2] + oz;
                            const int cy = pos[1] + oy - cy0;
                            if (L >= z0 && L < z1 && cy >= 0 && cy < kTile) {
                                float *ab = acc + (L & 1) * kTile * kTile * CP + cy * kTile * CP + iz * N1 * N1 +
                                            iy * N1;
                                if constexpr (N1 % 4 == 0) {
                                    if (4 * q < N) {
                                        const int ox = (4 * q) / N1, ix = (4 * q) % N1;
                                        const int cx = pos[0] + ox - cx0;
                                        if (cx >= 0 && cx < kTile) {
                                            float4 *ap = reinterpret_cast<float4 *>(ab + cx * CP + ix);
                                            float4 a4 = *ap;
                                            a4.x += Fs * C[0];
                                            a4.y += Fs * C[1];
                                            a4.z += Fs * C[2];
                                            a4.w += Fs * C[3];
                                            *ap = a4;
                                        }
                                    }
                                } else {
#pragma unroll
                                    for (int i = 0; i < 4; ++i) {
                                        const int a0 = 4 * q + i;
                                        if (a0 < N) {
                                            const int cx = pos[0] + a0 / N1 - cx0;
                                            if (cx >= 0 && cx < kTile) ab[cx * CP + a0 % N1] += Fs * C[i];
                                        }
                                    }
                                }
                            }
                        }
                    }
            }
            __syncthreads();  // the next round's patches share cells with this round's
        }
        if (vz - 1 >= z0 && vz - 1 < z1) flush(vz - 1);
        __syncthreads();
    }
    if (vz_hi == m2 - 1 && vz_hi >= z0 && vz_hi < z1) flush(vz_hi);
}

template <int N1, typename TR>
static fts_status launch_tile(const fts_level *lv, const fts_eigs *eg, float omega, int bf, const TR *r, double *x,
                              hipStream_t st) {
    TileGrid tg{};
    tg.nt[0] = (lv->m[0] + kTile - 1) / kTile;
    tg.nt[1] = (lv->m[1] + kTile - 1) / kTile;
    const int ntxy = tg.nt[0] * tg.nt[1];
    // segments along z: enough workgroups for four per compute unit
    tg.nseg = std::max(1, std::min(lv->m[2], (1024 + ntxy - 1) / ntxy));
    tg.zlen = (lv->m[2] + tg.nseg - 1) / tg.nseg;
    tg.nseg = (lv->m[2] + tg.zlen - 1) / tg.zlen;
    tg.ntile = ntxy * tg.nseg;
    tg.per_xcd = (tg.ntile + 7) / 8;
    const dim3 grid((unsigned)(8 * tg.per_xcd)), block(256);
    if (bf)
        k_schwarz_mfma_tile<N1, 1, TR><<<grid, block, 0, st>>>(lv->view, eg->view, tg, r, x, omega);
    else
        k_schwarz_mfma_tile<N1, 0, TR><<<grid, block, 0, st>>>(lv->view, eg->view, tg, r, x, omega);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FTS_OK : hip_fail(e, "k_schwarz_mfma_tile launch");
}

fts_status launch_schwarz_mfma_tile(const fts_level *lv, const fts_eigs *eg, double omega, int bf, const void *r,
                                    bool r_f32, double *x, hipStream_t st) {
    if (lv->dim != 3 || eg->kind != FTS_VERTEX_PATCH)
        return fail(FTS_E_UNSUPPORTED, "owner tiles: 3-D vertex patches only");
    if ((int64_t)lv->m[0] * lv->m[1] * lv->m[2] > INT_MAX) return fail(FTS_E_SIZE, "owner tiles: too many cells");
    const float om = (float)omega;
    const double *rd = static_cast<const double *>(r);
    const float *rf = static_cast<const float *>(r);
#define FTS_TILE_CASE(n)                                                                           \
    case n:                                                                                        \
        return r_f32 ? launch_tile<n>(lv, eg, om, bf, rf, x, st) : launch_tile<n>(lv, eg, om, bf, rd, x, st);
    switch (lv->n1) {
        FTS_TILE_CASE(2)
        FTS_TILE_CASE(3)
        FTS_TILE_CASE(4)
        FTS_TILE_CASE(5)
        FTS_TILE_CASE(6)
        FTS_TILE_CASE(7)
        FTS_TILE_CASE(8)
        default: return fail(FTS_E_UNSUPPORTED, "owner tiles: 16-bit MFMA contractions need n <= 16");
    }
#undef FTS_TILE_CASE
}

}  // namespace fts
