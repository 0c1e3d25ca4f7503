// Meshes of mapped (non-Cartesian) cells and the Cartesian surrogate local
// solvers of Sec. 4: the matrix-free SIPG operator on multilinearly mapped
// cells and the additive cell smoother whose local solvers are the
// fast-diagonalisation inverses of rectangular surrogate cells
// (eq. schwarzproj, eq. avglength).
//
// Geometry: a logically Cartesian mesh, cell c = image of [0, 1]^d under the
// multilinear map through its 2^d vertices.  The operator is eq. (bfsipg)
// with grad phi = J^-T grad_xi phi, volume element det J, face normal
// n = J^-T e_t / |J^-T e_t| and area element det J |J^-T e_t| (Nanson),
// evaluated by the (k+1)-point Gauss rule per axis on cells and faces; the
// penalty's h+- orthogonal to a face is |K| / |F|.  One workgroup per cell;
// every tensor of a cell (values, reference gradients, fluxes) lives in LDS
// and each 1-D contraction is one pass over the output tensor.
#include <algorithm>
#include <cmath>

#include "device_common.h"

namespace fts {

struct MappedView {
    int m[3];
    int64_t ncells;
    const double *verts;  // prod(m + 1) x dim vertex coordinates, x fastest
    const double *V, *D;  // n1 x n1: phi_i and phi_i' at the Gauss points [q][i]
    const double *xq, *wq;  // n1 Gauss points and weights on [0, 1]
    const double *dend;   // 2 x n1: phi_i'(0), phi_i'(1)
    const double *pen;    // ncells x 2d: penalty coefficient of face (t, side) at 2t + side
    const double *S;      // ncells x d x n1 x n1: surrogate eigenvectors, row-major [i][m]
    const double *lam;    // ncells x d x n1: surrogate eigenvalues
};

}  // namespace fts

struct fts_mapped_level {
    int dim = 0, k = 0, n1 = 0;
    int m[3] = {1, 1, 1};
    double gamma_hat = 1.0;
    int64_t ncells = 0, ndofs = 0;
    std::vector<double> hbar;  // surrogate widths, ncells x dim
    double *d_tab = nullptr;
    fts::MappedView view{};
};

namespace fts {

constexpr int kMapThreads = 64;

// out = contraction of the tensor `in` (extents e[0..D-1], x fastest) along
// axis a with the matrix M: out[.., o, ..] = sum_i M(o, i) in[.., i, ..], where
// M(o, i) = M[o * ld + i] (trans = false) or M[i * ld + o] (trans = true); the
// output extent along a is nout.  acc: add to out.  Ends with a barrier.
template <int D>
__device__ void contract(const double *in, const int *e, int a, const double *M, int ld, bool trans, int nout,
                         double *out, bool acc) {
    int eo[3] = {1, 1, 1};
    for (int b = 0; b < D; ++b) eo[b] = e[b];
    eo[a] = nout;
    const int total = eo[0] * eo[1] * eo[2];
    int stride_in = 1;
    for (int b = 0; b < a; ++b) stride_in *= e[b];
    for (int p = threadIdx.x; p < total; p += blockDim.x) {
        int o[3] = {p % eo[0], (p / eo[0]) % eo[1], p / (eo[0] * eo[1])};
        const int oa = o[a];
        o[a] = 0;
        const int base = o[0] + e[0] * (o[1] + e[1] * o[2]);
        double s = 0.0;
        for (int i = 0; i < e[a]; ++i) s += (trans ? M[i * ld + oa] : M[oa * ld + i]) * in[base + i * stride_in];
        out[p] = acc ? out[p] + s : s;
    }
    __syncthreads();
}

// Jacobian J[b][a] = d x_b / d xi_a of the multilinear map through the corners
// X[corner * D + b] (corner = sum_a o_a 2^a) at xi; returns det J and J^-1.
// The loop over the corners is unrolled UNR times.  Fully unrolled, the 3-D
// operator kernel loads all 24 corner coordinates at once and the two
// Jacobians of a face point hold about 200 VGPRs (two waves per SIMD); four
// corners at a time keep it near 96 (five waves), which is faster for
// k <= 4 (32^3 Q3 distorted residual 0.44 -> 0.31 ms).  For k >= 5 LDS caps
// the occupancy at three waves anyway and the full unroll is faster (16^3 Q5:
// 0.134 against 0.147 ms).
template <int D, int UNR = (1 << D)>
__device__ double jacobian_inverse(const double *X, const double *xi, double Ji[D][D]) {
    double J[D][D];
    for (int b = 0; b < D; ++b)
        for (int a = 0; a < D; ++a) J[b][a] = 0.0;
#pragma unroll UNR
    for (int cidx = 0; cidx < (1 << D); ++cidx)
        for (int a = 0; a < D; ++a) {
            double dN = ((cidx >> a) & 1) ? 1.0 : -1.0;
            for (int a2 = 0; a2 < D; ++a2)
                if (a2 != a) dN *= ((cidx >> a2) & 1) ? xi[a2] : 1.0 - xi[a2];
            for (int b = 0; b < D; ++b) J[b][a] += dN * X[cidx * D + b];
        }
    double det;
    if constexpr (D == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double id = 1.0 / det;
        Ji[0][0] = J[1][1] * id;
        Ji[0][1] = -J[0][1] * id;
        Ji[1][0] = -J[1][0] * id;
        Ji[1][1] = J[0][0] * id;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double id = 1.0 / det;
        Ji[0][0] = c00 * id;
        Ji[1][0] = c01 * id;
        Ji[2][0] = c02 * id;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    }
    return det;
}

// Corners per step of the Jacobian's corner loop for degree N1 - 1.
template <int D, int N1>
constexpr int jac_unroll() { return (D == 3 && N1 <= 5) ? 4 : (1 << D); }

template <int D>
__device__ void load_corners(const MappedView &g, int64_t cell, double *X) {
    int c[3] = {(int)(cell % g.m[0]), (int)((cell / g.m[0]) % g.m[1]), (int)(cell / ((int64_t)g.m[0] * g.m[1]))};
    for (int e2 = threadIdx.x; e2 < (1 << D) * D; e2 += blockDim.x) {
        const int cidx = e2 / D, b = e2 % D;
        int v[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) v[a] = c[a] + ((cidx >> a) & 1);
        const int64_t vi = v[0] + (int64_t)(g.m[0] + 1) * (v[1] + (int64_t)(g.m[1] + 1) * v[2]);
        X[e2] = g.verts[vi * D + b];
    }
}

// Layout of the face work arrays (doubles) inside the kernel's work buffer,
// NF = points of a face: value and normal-derivative node layers of both
// sides [sd][kind][NF], the first tangential stage [sd][3][NF], values and
// reference gradients at the face's Gauss points [sd][NF], [sd][D][NF], the
// test coefficients [NF], [D][NF], the first stage of their test [4][NF] and
// the layer sums [NF] x 2.
template <int D, int NF>
struct FaceWork {
    static constexpr int LAY = 0, S1 = LAY + 4 * NF, FV = S1 + 6 * NF, FG = FV + 2 * NF, CV = FG + 2 * D * NF,
                         CG = CV + NF, S2 = CG + D * NF, LT = S2 + 4 * NF, T2T = LT + NF, SIZE = T2T + NF;
};

// The terms of face (TT, SIDE) of one cell, added to Y: traces of u and of the
// neighbour's u at the face's Gauss points (node layer at the face and normal
// derivative layer, then interpolation along the tangential axes TA, TB),
// the pointwise SIPG integrands (jump, average normal flux, penalty) and
// their test against the cell's basis.  Every stage is one pass over all of
// its outputs (both sides, all quantities) and ends with a barrier.
template <int D, int N1, int TT, int SIDE>
__device__ __forceinline__ void face_terms(const MappedView &g, int64_t cell, const int *cc,
                                           const double *__restrict__ x, const double *U, double *Un,
                                           const double *X, double *Xn, const double *sV, const double *sD,
                                           const double *sxq, const double *swq, const double *sde, double *work,
                                           double *Y) {
    constexpr int NC = D == 2 ? N1 * N1 : N1 * N1 * N1;
    constexpr int NF = D == 2 ? N1 : N1 * N1;
    constexpr int TA = TT == 0 ? 1 : 0, TB = D == 3 ? (TT == 2 ? 1 : 2) : 0;
    using W = FaceWork<D, NF>;
    double *Lay = work + W::LAY, *S1 = work + W::S1, *Fv = work + W::FV, *Fg = work + W::FG, *Cv = work + W::CV,
           *Cg = work + W::CG, *S2 = work + W::S2, *Lt = work + W::LT, *T2t = work + W::T2T;
    const int t = threadIdx.x, nth = blockDim.x;
    // index in the cell tensor of node it along TT, ia along TA, ib along TB
    auto cidx = [](int it, int ia, int ib) {
        int o[3] = {0, 0, 0};
        o[TT] = it;
        o[TA] = ia;
        if constexpr (D == 3) o[TB] = ib;
        return o[0] + N1 * (o[1] + N1 * o[2]);
    };
    const bool interior = SIDE == 0 ? cc[TT] > 0 : cc[TT] < g.m[TT] - 1;
    if (interior) {
        int64_t st = 1;
        for (int a = 0; a < TT; ++a) st *= g.m[a];
        const int64_t nb = cell + (SIDE == 0 ? -st : st);
        load_corners<D>(g, nb, Xn);
        for (int e = t; e < NC; e += nth) Un[e] = x[nb * NC + e];
        __syncthreads();
    }
    const int nsd = interior ? 2 : 1;
    // node layers: value at the face's node layer and normal derivative
    for (int e = t; e < nsd * 2 * NF; e += nth) {
        const int sd = e / (2 * NF), kind = (e / NF) % 2, lp = e % NF;
        const int ia = lp % N1, ib = lp / N1;
        const double *Us = sd ? Un : U;
        const int sh = sd ? 1 - SIDE : SIDE;
        double v;
        if (kind == 0) {
            v = Us[cidx(sh * (N1 - 1), ia, ib)];
        } else {
            v = 0.0;
#pragma unroll
            for (int i = 0; i < N1; ++i) v += sde[sh * N1 + i] * Us[cidx(i, ia, ib)];
        }
        Lay[(sd * 2 + kind) * NF + lp] = v;
    }
    __syncthreads();
    // along TA: V (values), V (normal derivative), D (tangential derivative along TA)
    for (int e = t; e < nsd * 3 * NF; e += nth) {
        const int sd = e / (3 * NF), out = (e / NF) % 3, r = e % NF;
        const int ga = r % N1, ib = r / N1;
        const double *M = out == 2 ? sD : sV;
        const double *src = Lay + (sd * 2 + (out == 1 ? 1 : 0)) * NF + N1 * ib;
        double v = 0.0;
#pragma unroll
        for (int ia = 0; ia < N1; ++ia) v += M[ga * N1 + ia] * src[ia];
        if constexpr (D == 2) {
            double *dst = out == 0 ? Fv + sd * NF : Fg + (sd * D + (out == 1 ? TT : TA)) * NF;
            dst[r] = v;
        } else {
            S1[(sd * 3 + out) * NF + r] = v;
        }
    }
    __syncthreads();
    if constexpr (D == 3) {
        // along TB: values, normal derivative, derivative along TA, derivative along TB
        for (int e = t; e < nsd * 4 * NF; e += nth) {
            const int sd = e / (4 * NF), out = (e / NF) % 4, p = e % NF;
            const int ga = p % N1, gb = p / N1;
            const double *M = out == 3 ? sD : sV;
            const double *src = S1 + (sd * 3 + (out == 3 ? 0 : out)) * NF + ga;
            double v = 0.0;
#pragma unroll
            for (int ib = 0; ib < N1; ++ib) v += M[gb * N1 + ib] * src[N1 * ib];
            double *dst = out == 0 ? Fv + sd * NF : Fg + (sd * D + (out == 1 ? TT : (out == 2 ? TA : TB))) * NF;
            dst[p] = v;
        }
        __syncthreads();
    }
    // pointwise face terms: coefficients of phi_i and of grad_xi phi_i
    const double pen = g.pen[cell * 2 * D + 2 * TT + SIDE];
    for (int p = t; p < NF; p += nth) {
        const int ga = p % N1, gb = p / N1;
        double xi[D], xin[D];
        xi[TT] = SIDE;
        xin[TT] = 1 - SIDE;
        xi[TA] = xin[TA] = sxq[ga];
        double wf = swq[ga];
        if constexpr (D == 3) {
            xi[TB] = xin[TB] = sxq[gb];
            wf *= swq[gb];
        }
        double Ji[D][D];
        const double det = jacobian_inverse<D, jac_unroll<D, N1>()>(X, xi, Ji);
        double nrm = 0.0;
        for (int b = 0; b < D; ++b) nrm += Ji[TT][b] * Ji[TT][b];
        nrm = sqrt(nrm);
        const double sgn = SIDE ? 1.0 : -1.0;
        double n[D];
        for (int b = 0; b < D; ++b) n[b] = sgn * Ji[TT][b] / nrm;
        const double dS = wf * fabs(det) * nrm;
        double dnm = 0.0;  // normal derivative of u on this side
        for (int b = 0; b < D; ++b) {
            double ph = 0.0;
            for (int a = 0; a < D; ++a) ph += Ji[a][b] * Fg[a * NF + p];
            dnm += ph * n[b];
        }
        double cv, jmp;
        if (interior) {
            double Jn[D][D];
            (void)jacobian_inverse<D, jac_unroll<D, N1>()>(Xn, xin, Jn);
            double dnp = 0.0;
            for (int b = 0; b < D; ++b) {
                double ph = 0.0;
                for (int a = 0; a < D; ++a) ph += Jn[a][b] * Fg[(D + a) * NF + p];
                dnp += ph * n[b];
            }
            jmp = Fv[p] - Fv[NF + p];
            cv = dS * (pen * jmp - 0.5 * (dnm + dnp));
            jmp *= 0.5;
        } else {
            jmp = Fv[p];
            cv = dS * (pen * jmp - dnm);
        }
        // - jmp dS n . grad phi_i = grad_xi phi_i . (J^-1 (-jmp dS n))
        Cv[p] = cv;
        for (int a = 0; a < D; ++a) {
            double s2 = 0.0;
            for (int b = 0; b < D; ++b) s2 += Ji[a][b] * n[b];
            Cg[a * NF + p] = -jmp * dS * s2;
        }
    }
    __syncthreads();
    // test, along TA (transposed): value and tangential-gradient terms land on
    // the node layer of the face, the normal-gradient term spreads over the
    // layers with phi_i'(SIDE)
    if constexpr (D == 2) {
        for (int e = t; e < 2 * N1; e += nth) {
            const int out = e / N1, ia = e % N1;
            double v = 0.0;
            if (out == 0) {
#pragma unroll
                for (int ga = 0; ga < N1; ++ga) v += sV[ga * N1 + ia] * Cv[ga] + sD[ga * N1 + ia] * Cg[TA * NF + ga];
                Lt[ia] = v;
            } else {
#pragma unroll
                for (int ga = 0; ga < N1; ++ga) v += sV[ga * N1 + ia] * Cg[TT * NF + ga];
                T2t[ia] = v;
            }
        }
        __syncthreads();
    } else {
        for (int e = t; e < 4 * NF; e += nth) {
            const int out = e / NF, r = e % NF;
            const int ia = r % N1, gb = r / N1;
            const double *M = out == 1 ? sD : sV;
            const double *src = (out == 0 ? Cv : Cg + (out == 1 ? TA : (out == 2 ? TB : TT)) * NF) + N1 * gb;
            double v = 0.0;
#pragma unroll
            for (int ga = 0; ga < N1; ++ga) v += M[ga * N1 + ia] * src[ga];
            S2[out * NF + r] = v;
        }
        __syncthreads();
        for (int e = t; e < 2 * NF; e += nth) {
            const int out = e / NF, r = e % NF;
            const int ia = r % N1, ib = r / N1;
            double v = 0.0;
            if (out == 0) {
#pragma unroll
                for (int gb = 0; gb < N1; ++gb) {
                    const int q = ia + N1 * gb;
                    v += sV[gb * N1 + ib] * (S2[q] + S2[NF + q]) + sD[gb * N1 + ib] * S2[2 * NF + q];
                }
                Lt[r] = v;
            } else {
#pragma unroll
                for (int gb = 0; gb < N1; ++gb) v += sV[gb * N1 + ib] * S2[3 * NF + ia + N1 * gb];
                T2t[r] = v;
            }
        }
        __syncthreads();
    }
    for (int p = t; p < NC; p += nth) {
        int o[3] = {p % N1, (p / N1) % N1, p / (N1 * N1)};
        const int it = o[TT];
        const int lp = o[TA] + (D == 3 ? N1 * o[TB] : 0);
        double add = sde[SIDE * N1 + it] * T2t[lp];
        if (it == SIDE * (N1 - 1)) add += Lt[lp];
        Y[p] += add;
    }
    __syncthreads();
}

// y = A x (or r = b - A x) on every cell; grid = ncells, one cell per workgroup.
template <int D, int N1, bool RES>
__global__ void __launch_bounds__(kMapThreads)
k_mapped_operator(MappedView g, const double *__restrict__ x, const double *__restrict__ bvec,
                  double *__restrict__ y) {
    constexpr int NC = D == 2 ? N1 * N1 : N1 * N1 * N1;
    constexpr int NF = D == 2 ? N1 : N1 * N1;  // points of a face
    __shared__ double sV[N1 * N1], sD[N1 * N1], sxq[N1], swq[N1], sde[2 * N1];
    __shared__ double X[8 * 3], Xn[8 * 3];
    __shared__ double U[NC], Un[NC], Y[NC];
    // volume stage: T1, T2 and the reference gradients / fluxes G[0..D-1];
    // then the face stages (FaceWork)
    constexpr int NW = 5 * NC > FaceWork<D, NF>::SIZE ? 5 * NC : FaceWork<D, NF>::SIZE;
    __shared__ double work[NW];
    double *T1 = work, *T2 = work + NC;
    auto G = [&](int a) { return work + (2 + a) * NC; };
    const int64_t cell = blockIdx.x;
    const int t = threadIdx.x;
    for (int e2 = t; e2 < N1 * N1; e2 += blockDim.x) {
        sV[e2] = g.V[e2];
        sD[e2] = g.D[e2];
    }
    for (int e2 = t; e2 < N1; e2 += blockDim.x) {
        sxq[e2] = g.xq[e2];
        swq[e2] = g.wq[e2];
        sde[e2] = g.dend[e2];
        sde[N1 + e2] = g.dend[N1 + e2];
    }
    load_corners<D>(g, cell, X);
    for (int e2 = t; e2 < NC; e2 += blockDim.x) {
        U[e2] = x[cell * NC + e2];
        Y[e2] = 0.0;
    }
    __syncthreads();
    const int ec[3] = {N1, N1, D == 3 ? N1 : 1};

    // ---- volume: grad_xi u at the Gauss points, flux w det J J^-1 J^-T grad_xi u, test
    for (int a = 0; a < D; ++a) {
        contract<D>(U, ec, 0, a == 0 ? sD : sV, N1, false, N1, T1, false);
        if constexpr (D == 2) {
            contract<D>(T1, ec, 1, a == 1 ? sD : sV, N1, false, N1, G(a), false);
        } else {
            contract<D>(T1, ec, 1, a == 1 ? sD : sV, N1, false, N1, T2, false);
            contract<D>(T2, ec, 2, a == 2 ? sD : sV, N1, false, N1, G(a), false);
        }
    }
    for (int p = t; p < NC; p += blockDim.x) {
        const int q[3] = {p % N1, (p / N1) % N1, p / (N1 * N1)};
        double xi[D], w = 1.0;
        for (int a = 0; a < D; ++a) {
            xi[a] = sxq[q[a]];
            w *= swq[q[a]];
        }
        double Ji[D][D];
        const double det = jacobian_inverse<D, jac_unroll<D, N1>()>(X, xi, Ji);
        double gr[D], fl[D];
        for (int a = 0; a < D; ++a) gr[a] = G(a)[p];
        // physical gradient J^-T gr, then back: flux_a = w det sum_b Ji[a][b] (J^-T gr)_b
        double ph[D];
        for (int b = 0; b < D; ++b) {
            ph[b] = 0.0;
            for (int a = 0; a < D; ++a) ph[b] += Ji[a][b] * gr[a];
        }
        for (int a = 0; a < D; ++a) {
            fl[a] = 0.0;
            for (int b = 0; b < D; ++b) fl[a] += Ji[a][b] * ph[b];
            fl[a] *= w * det;
        }
        for (int a = 0; a < D; ++a) G(a)[p] = fl[a];
    }
    __syncthreads();
    for (int a = 0; a < D; ++a) {
        if constexpr (D == 2) {
            contract<D>(G(a), ec, 0, a == 0 ? sD : sV, N1, true, N1, T1, false);
            contract<D>(T1, ec, 1, a == 1 ? sD : sV, N1, true, N1, Y, true);
        } else {
            contract<D>(G(a), ec, 0, a == 0 ? sD : sV, N1, true, N1, T1, false);
            contract<D>(T1, ec, 1, a == 1 ? sD : sV, N1, true, N1, T2, false);
            contract<D>(T2, ec, 2, a == 2 ? sD : sV, N1, true, N1, Y, true);
        }
    }

    // ---- faces, one after the other (fixed order: axis, then lower and upper side)
    const int cc[3] = {(int)(cell % g.m[0]), (int)((cell / g.m[0]) % g.m[1]),
                       (int)(cell / ((int64_t)g.m[0] * g.m[1]))};
#define FTS_FACE(TT, SIDE) \
    face_terms<D, N1, TT, SIDE>(g, cell, cc, x, U, Un, X, Xn, sV, sD, sxq, swq, sde, work, Y);
    FTS_FACE(0, 0)
    FTS_FACE(0, 1)
    FTS_FACE(1, 0)
    FTS_FACE(1, 1)
    if constexpr (D == 3) {
        FTS_FACE(2, 0)
        FTS_FACE(2, 1)
    }
#undef FTS_FACE
    for (int e2 = t; e2 < NC; e2 += blockDim.x) {
        const int64_t gi = cell * NC + e2;
        y[gi] = RES ? bvec[gi] - Y[e2] : Y[e2];
    }
}

// Red-black color of cell c (x fastest, m0 x m1 cells per layer): the parity
// of its index sum.  Face neighbours have opposite colors.
__device__ __forceinline__ int cell_parity(int dim, int m0, int m1, int64_t c) {
    const int64_t c1 = c / m0;
    const int64_t sum = c % m0 + (dim == 3 ? c1 % m1 + c1 / m1 : c1);
    return (int)(sum & 1);
}

// x += omega sum_K R_K^T Atilde_K^-1 R_K r with the surrogate tables of each
// cell: (S_d x .. x S_1) diag(1 / sum_t lambda_t) (S_d x .. x S_1)^T.
// color >= 0: only the cells whose index sum has that parity (the red-black
// coloring of the multiplicative smoother); the others leave at once.
template <int D, int N1>
__global__ void __launch_bounds__(kMapThreads)
k_mapped_surrogate(MappedView g, double omega, int color, const double *__restrict__ r, double *__restrict__ x) {
    constexpr int NC = D == 2 ? N1 * N1 : N1 * N1 * N1;
    __shared__ double A[NC], B[NC];
    __shared__ double S[D][N1 * N1], L[D][N1];
    const int64_t cell = blockIdx.x;
    // uniform over the workgroup: it leaves before any barrier
    if (color >= 0 && cell_parity(D, g.m[0], g.m[1], cell) != color) return;
    const int t = threadIdx.x;
    for (int e2 = t; e2 < D * N1 * N1; e2 += blockDim.x) S[e2 / (N1 * N1)][e2 % (N1 * N1)] = g.S[cell * D * N1 * N1 + e2];
    for (int e2 = t; e2 < D * N1; e2 += blockDim.x) L[e2 / N1][e2 % N1] = g.lam[cell * D * N1 + e2];
    for (int e2 = t; e2 < NC; e2 += blockDim.x) A[e2] = r[cell * NC + e2];
    __syncthreads();
    const int ec[3] = {N1, N1, D == 3 ? N1 : 1};
    // forward: out_m = sum_i S[i][m] in_i along every axis
    contract<D>(A, ec, 0, S[0], N1, true, N1, B, false);
    contract<D>(B, ec, 1, S[1], N1, true, N1, A, false);
    double *cur = A, *oth = B;
    if constexpr (D == 3) {
        contract<D>(A, ec, 2, S[2], N1, true, N1, B, false);
        cur = B;
        oth = A;
    }
    for (int p = t; p < NC; p += blockDim.x) {
        const int m[3] = {p % N1, (p / N1) % N1, p / (N1 * N1)};
        double lam = 0.0;
        for (int a = 0; a < D; ++a) lam += L[a][m[a]];
        cur[p] *= omega / lam;
    }
    __syncthreads();
    // backward: out_i = sum_m S[i][m] in_m
    contract<D>(cur, ec, 0, S[0], N1, false, N1, oth, false);
    contract<D>(oth, ec, 1, S[1], N1, false, N1, cur, false);
    double *res = cur;
    if constexpr (D == 3) {
        contract<D>(cur, ec, 2, S[2], N1, false, N1, oth, false);
        res = oth;
    }
    for (int e2 = t; e2 < NC; e2 += blockDim.x) x[cell * NC + e2] += res[e2];
}

template <int D, int N1>
static fts_status launch_mapped_op(const fts_mapped_level *lv, const double *x, const double *b, double *y,
                                   bool res, hipStream_t st) {
    const dim3 grid((unsigned)lv->ncells), block(kMapThreads);
    if (res)
        k_mapped_operator<D, N1, true><<<grid, block, 0, st>>>(lv->view, x, b, y);
    else
        k_mapped_operator<D, N1, false><<<grid, block, 0, st>>>(lv->view, x, b, y);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FTS_OK : hip_fail(e, "k_mapped_operator launch");
}

template <int D, int N1>
static fts_status launch_mapped_sur(const fts_mapped_level *lv, double omega, int color, const double *r, double *x,
                                    hipStream_t st) {
    k_mapped_surrogate<D, N1><<<dim3((unsigned)lv->ncells), dim3(kMapThreads), 0, st>>>(lv->view, omega, color, r,
                                                                                          x);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FTS_OK : hip_fail(e, "k_mapped_surrogate launch");
}

// Largest N1 = k + 1 on mapped cells: k <= 7 in 3-D (the cell's work arrays
// stay in LDS at several workgroups per CU), k <= 15 in 2-D.
template <int D>
constexpr int map_max_n1() { return D == 2 ? 16 : 8; }

template <int D, int N1 = 2>
static fts_status dispatch_mapped(const fts_mapped_level *lv, int what, double omega, int color, const double *x,
                                  const double *b, double *y, hipStream_t st) {
    if constexpr (N1 > map_max_n1<D>()) {
        return fail(FTS_E_UNSUPPORTED, "mapped meshes: degree above 7 in 3-D or 15 in 2-D");
    } else {
        if (lv->n1 != N1) return dispatch_mapped<D, N1 + 1>(lv, what, omega, color, x, b, y, st);
        if (what == 2) return launch_mapped_sur<D, N1>(lv, omega, color, x, y, st);
        return launch_mapped_op<D, N1>(lv, x, b, y, what == 1, st);
    }
}

// what: 0 y = A x, 1 y = b - A x, 2 y += omega (surrogate solves) x over all
// cells (color < 0) or over one red-black color.
static fts_status run_mapped(const fts_mapped_level *lv, int what, double omega, const double *x, const double *b,
                             double *y, hipStream_t st, int color = -1) {
    if (lv->ncells == 0) return FTS_OK;
    return lv->dim == 2 ? dispatch_mapped<2>(lv, what, omega, color, x, b, y, st)
                        : dispatch_mapped<3>(lv, what, omega, color, x, b, y, st);
}

// ---- host geometry (FP64): multilinear map, cell volumes, face areas
static void host_jacobian(int d, const double *X, const double *xi, double *J) {
    for (int i = 0; i < d * d; ++i) J[i] = 0.0;
    for (int cidx = 0; cidx < (1 << d); ++cidx)
        for (int a = 0; a < d; ++a) {
            double dN = ((cidx >> a) & 1) ? 1.0 : -1.0;
            for (int a2 = 0; a2 < d; ++a2)
                if (a2 != a) dN *= ((cidx >> a2) & 1) ? xi[a2] : 1.0 - xi[a2];
            for (int b = 0; b < d; ++b) J[b * d + a] += dN * X[cidx * d + b];
        }
}

static double host_det_inv(int d, const double *J, double *Ji) {
    if (d == 2) {
        const double det = J[0] * J[3] - J[1] * J[2];
        Ji[0] = J[3] / det;
        Ji[1] = -J[1] / det;
        Ji[2] = -J[2] / det;
        Ji[3] = J[0] / det;
        return det;
    }
    const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
    const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
    Ji[0] = c00 / det;
    Ji[3] = c01 / det;
    Ji[6] = c02 / det;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

}  // namespace fts

using namespace fts;

extern "C" {

fts_status fts_mapped_level_create(const fts_mapped_desc *desc, fts_mapped_level **out) {
    if (!desc || !out || !desc->vertices) return fail(FTS_E_INVAL, "fts_mapped_level_create: NULL argument");
    *out = nullptr;
    const int d = desc->dim;
    if (d != 2 && d != 3) return fail(FTS_E_UNSUPPORTED, "mapped meshes: dim must be 2 or 3");
    if (desc->degree < 1 || desc->degree > (d == 2 ? map_max_n1<2>() : map_max_n1<3>()) - 1)
        return fail(FTS_E_UNSUPPORTED, "mapped meshes: degree must be in 1..7 (3-D) or 1..15 (2-D)");
    if (!(desc->penalty_factor > 0.0) || !std::isfinite(desc->penalty_factor))
        return fail(FTS_E_INVAL, "penalty_factor must be positive");
    auto *lv = new fts_mapped_level();
    lv->dim = d;
    lv->k = desc->degree;
    lv->n1 = desc->degree + 1;
    lv->gamma_hat = desc->penalty_factor;
    lv->ncells = 1;
    int64_t nverts = 1;
    for (int a = 0; a < 3; ++a) {
        lv->m[a] = a < d ? desc->ncells[a] : 1;
        if (lv->m[a] < 1) {
            delete lv;
            return fail(FTS_E_INVAL, "ncells must be >= 1");
        }
        lv->ncells *= lv->m[a];
        if (a < d) nverts *= lv->m[a] + 1;
    }
    const int n1 = lv->n1, nc = d == 2 ? n1 * n1 : n1 * n1 * n1;
    lv->ndofs = lv->ncells * nc;
    const double *V0 = desc->vertices;
    for (int64_t i = 0; i < nverts * d; ++i)
        if (!std::isfinite(V0[i])) {
            delete lv;
            return fail(FTS_E_INVAL, "vertex coordinates must be finite");
        }
    std::vector<double> xq, wq, Vb, Db;
    gauss_basis(lv->k, xq, wq, Vb, Db);
    Ref1D ref;
    ref.build(lv->k);
    const int64_t nce = lv->ncells;
    auto corners = [&](int64_t cell, double *X) {
        const int c[3] = {(int)(cell % lv->m[0]), (int)((cell / lv->m[0]) % lv->m[1]),
                          (int)(cell / ((int64_t)lv->m[0] * lv->m[1]))};
        for (int cidx = 0; cidx < (1 << d); ++cidx) {
            int v[3] = {0, 0, 0};
            for (int a = 0; a < d; ++a) v[a] = c[a] + ((cidx >> a) & 1);
            const int64_t vi = v[0] + (int64_t)(lv->m[0] + 1) * (v[1] + (int64_t)(lv->m[1] + 1) * v[2]);
            for (int b = 0; b < d; ++b) X[cidx * d + b] = V0[vi * d + b];
        }
    };
    // cell volumes and face areas (the face between a cell and its upper
    // neighbour is measured from the lower cell; boundary faces from their cell)
    std::vector<double> vol(nce), area(nce * 2 * d, 0.0);
    double X[24], J[9], Ji[9];
    for (int64_t cell = 0; cell < nce; ++cell) {
        corners(cell, X);
        double v = 0.0;
        for (int p = 0; p < nc; ++p) {
            const int q[3] = {p % n1, (p / n1) % n1, p / (n1 * n1)};
            double xi[3], w = 1.0;
            for (int a = 0; a < d; ++a) {
                xi[a] = xq[q[a]];
                w *= wq[q[a]];
            }
            host_jacobian(d, X, xi, J);
            const double det = host_det_inv(d, J, Ji);
            if (!(det > 0.0)) {
                delete lv;
                return fail(FTS_E_INVAL, "a cell map is not orientation preserving (det J <= 0)");
            }
            v += w * det;
        }
        vol[cell] = v;
        for (int t = 0; t < d; ++t)
            for (int side = 0; side < 2; ++side) {
                double A = 0.0;
                const int nf = nc / n1;
                for (int p = 0; p < nf; ++p) {
                    int o[3] = {0, 0, 0}, r2 = p;
                    double xi[3], w = 1.0;
                    for (int a = 0; a < d; ++a) {
                        if (a == t) {
                            xi[a] = side;
                            continue;
                        }
                        o[a] = r2 % n1;
                        r2 /= n1;
                        xi[a] = xq[o[a]];
                        w *= wq[o[a]];
                    }
                    host_jacobian(d, X, xi, J);
                    const double det = host_det_inv(d, J, Ji);
                    double nrm = 0.0;
                    for (int b = 0; b < d; ++b) nrm += Ji[t * d + b] * Ji[t * d + b];
                    A += w * std::fabs(det) * std::sqrt(nrm);
                }
                area[cell * 2 * d + 2 * t + side] = A;
            }
    }
    // penalty coefficient of each face seen from each cell: gamma_e / 2 inside
    // (gamma_e = gamma_hat k (k+1) (1/h- + 1/h+), h = |K| / |F|), gamma_e on the boundary
    std::vector<double> pen(nce * 2 * d);
    const double gk = lv->gamma_hat * lv->k * (lv->k + 1.0);
    for (int64_t cell = 0; cell < nce; ++cell) {
        const int c[3] = {(int)(cell % lv->m[0]), (int)((cell / lv->m[0]) % lv->m[1]),
                          (int)(cell / ((int64_t)lv->m[0] * lv->m[1]))};
        int64_t st = 1;
        for (int t = 0; t < d; ++t) {
            for (int side = 0; side < 2; ++side) {
                const bool interior = side == 0 ? c[t] > 0 : c[t] < lv->m[t] - 1;
                double p;
                if (interior) {
                    const int64_t nb = cell + (side == 0 ? -st : st);
                    const int64_t lower = side == 0 ? nb : cell;
                    const double F = area[lower * 2 * d + 2 * t + 1];
                    p = 0.5 * gk * (F / vol[cell] + F / vol[nb]);
                } else {
                    p = gk * 2.0 * area[cell * 2 * d + 2 * t + side] / vol[cell];
                }
                pen[cell * 2 * d + 2 * t + side] = p;
            }
            st *= lv->m[t];
        }
    }
    // surrogate boxes (eq. avglength) and their 1-D eigenpairs per cell and axis
    lv->hbar.assign(nce * d, 0.0);
    for (int64_t cell = 0; cell < nce; ++cell) {
        corners(cell, X);
        for (int t = 0; t < d; ++t) {
            double s = 0.0;
            int cnt = 0;
            for (int cidx = 0; cidx < (1 << d); ++cidx) {
                if ((cidx >> t) & 1) continue;
                const int c2 = cidx | (1 << t);
                double l2 = 0.0;
                for (int b = 0; b < d; ++b) l2 += (X[c2 * d + b] - X[cidx * d + b]) * (X[c2 * d + b] - X[cidx * d + b]);
                s += std::sqrt(l2);
                ++cnt;
            }
            lv->hbar[cell * d + t] = s / cnt;
        }
    }
    std::vector<double> Sall(nce * d * n1 * n1), Lall(nce * d * n1);
    std::vector<double> A1(n1 * n1), M1(n1 * n1);
    for (int64_t cell = 0; cell < nce; ++cell) {
        const int c[3] = {(int)(cell % lv->m[0]), (int)((cell / lv->m[0]) % lv->m[1]),
                          (int)(cell / ((int64_t)lv->m[0] * lv->m[1]))};
        int64_t st = 1;
        for (int t = 0; t < d; ++t) {
            const double h = lv->hbar[cell * d + t];
            const double hl = c[t] > 0 ? lv->hbar[(cell - st) * d + t] : -1.0;
            const double hr = c[t] < lv->m[t] - 1 ? lv->hbar[(cell + st) * d + t] : -1.0;
            ref.cell_operator(h, hl, hr, lv->gamma_hat, A1.data());
            for (int i = 0; i < n1 * n1; ++i) M1[i] = h * ref.Mhat[i];
            const fts_status s2 = sym_gen_eig(n1, A1.data(), M1.data(), &Sall[(cell * d + t) * n1 * n1],
                                              &Lall[(cell * d + t) * n1]);
            if (s2 != FTS_OK) {
                delete lv;
                return s2;
            }
            st *= lv->m[t];
        }
    }
    // upload: vertices, V, D, xq, wq, end derivatives, penalties, S, lambda
    std::vector<double> dend(2 * n1);
    for (int i = 0; i < n1; ++i) {
        dend[i] = ref.d0[i];
        dend[n1 + i] = ref.d1[i];
    }
    const size_t sizes[9] = {(size_t)(nverts * d), (size_t)n1 * n1, (size_t)n1 * n1, (size_t)n1, (size_t)n1,
                             (size_t)2 * n1, pen.size(), Sall.size(), Lall.size()};
    const double *srcs[9] = {V0, Vb.data(), Db.data(), xq.data(), wq.data(), dend.data(), pen.data(), Sall.data(),
                             Lall.data()};
    size_t total = 0;
    for (size_t s2 : sizes) total += s2;
    if (dev_malloc(&lv->d_tab, total * sizeof(double)) != hipSuccess) {
        delete lv;
        return fail(FTS_E_HIP, "device allocation of the mapped-mesh tables failed");
    }
    const double *ptrs[9];
    size_t off = 0;
    for (int i = 0; i < 9; ++i) {
        if (hipMemcpy(lv->d_tab + off, srcs[i], sizes[i] * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
            dev_free(lv->d_tab);
            delete lv;
            return fail(FTS_E_HIP, "upload of the mapped-mesh tables failed");
        }
        ptrs[i] = lv->d_tab + off;
        off += sizes[i];
    }
    MappedView &vw = lv->view;
    for (int a = 0; a < 3; ++a) vw.m[a] = lv->m[a];
    vw.ncells = nce;
    vw.verts = ptrs[0];
    vw.V = ptrs[1];
    vw.D = ptrs[2];
    vw.xq = ptrs[3];
    vw.wq = ptrs[4];
    vw.dend = ptrs[5];
    vw.pen = ptrs[6];
    vw.S = ptrs[7];
    vw.lam = ptrs[8];
    *out = lv;
    return FTS_OK;
}

fts_status fts_mapped_level_destroy(fts_mapped_level *lv) {
    if (!lv) return FTS_OK;
    if (lv->d_tab) dev_free(lv->d_tab);
    delete lv;
    return FTS_OK;
}

int64_t fts_mapped_level_ndofs(const fts_mapped_level *lv) { return lv ? lv->ndofs : -1; }

fts_status fts_mapped_surrogate_widths(const fts_mapped_level *lv, double *hbar) {
    if (!lv || !hbar) return fail(FTS_E_INVAL, "fts_mapped_surrogate_widths: NULL argument");
    std::copy(lv->hbar.begin(), lv->hbar.end(), hbar);
    return FTS_OK;
}

fts_status fts_mapped_apply_operator(const fts_mapped_level *lv, const double *x, double *y, void *stream) {
    if (!lv || !x || !y) return fail(FTS_E_INVAL, "fts_mapped_apply_operator: NULL argument");
    if (x == y) return fail(FTS_E_INVAL, "fts_mapped_apply_operator: x and y must not alias");
    return run_mapped(lv, 0, 0.0, x, nullptr, y, reinterpret_cast<hipStream_t>(stream));
}

fts_status fts_mapped_residual(const fts_mapped_level *lv, const double *b, const double *x, double *r,
                               void *stream) {
    if (!lv || !b || !x || !r) return fail(FTS_E_INVAL, "fts_mapped_residual: NULL argument");
    if (r == x) return fail(FTS_E_INVAL, "fts_mapped_residual: r must not alias x");
    return run_mapped(lv, 1, 0.0, x, b, r, reinterpret_cast<hipStream_t>(stream));
}

fts_status fts_mapped_schwarz_apply(const fts_mapped_level *lv, double omega, const double *r, double *x,
                                    void *stream) {
    if (!lv || !r || !x) return fail(FTS_E_INVAL, "fts_mapped_schwarz_apply: NULL argument");
    if (r == x) return fail(FTS_E_INVAL, "fts_mapped_schwarz_apply: r and x must not alias");
    return run_mapped(lv, 2, omega, r, nullptr, x, reinterpret_cast<hipStream_t>(stream));
}

size_t fts_mapped_smooth_ws_bytes(const fts_mapped_level *lv) {
    return lv ? (size_t)lv->ndofs * sizeof(double) : 0;
}

fts_status fts_mapped_schwarz_smooth(const fts_mapped_level *lv, double omega, const double *b, double *x,
                                     int32_t nsweeps, void *ws, size_t ws_bytes, void *stream) {
    if (!lv || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_mapped_schwarz_smooth: NULL argument");
    if (ws_bytes < fts_mapped_smooth_ws_bytes(lv))
        return fail(FTS_E_SIZE, "fts_mapped_schwarz_smooth: workspace too small");
    double *r = static_cast<double *>(ws);
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int it = 0; it < nsweeps; ++it) {
        fts_status s = run_mapped(lv, 1, 0.0, x, b, r, st);
        if (s != FTS_OK) return s;
        s = run_mapped(lv, 2, omega, r, nullptr, x, st);
        if (s != FTS_OK) return s;
    }
    return FTS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Multigrid on mapped meshes (Sec. 4 with Alg. gmg): levels from uniform
// refinement on the cell maps, so the spaces are nested and the grid transfers
// are those of the Cartesian hierarchy in reference coordinates (embedding of
// the children, k_transfer); the additive cell smoother with the Cartesian
// surrogate local solvers on every level l >= 1; on level 0 the mapped
// operator's own matrix, probed column by column, factored by the slab LU of
// the Cartesian coarse solver.

namespace fts {

// e[(c, i)] = 1 for every cell c whose indices are congruent to col[] modulo
// 3 along every axis (two such cells are at least three apart along some axis,
// so no cell is a face neighbour, or itself, of two of them).
__global__ void k_probe_set(int dim, int m0, int m1, int64_t ncells, int nc, int col0, int col1, int col2, int i,
                            double *__restrict__ e) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const int cx = (int)(c % m0), r0 = (int)(c / m0);
        const int cy = dim == 3 ? r0 % m1 : r0, cz = dim == 3 ? r0 / m1 : 0;
        if (cx % 3 == col0 && cy % 3 == col1 && (dim == 2 || cz % 3 == col2)) e[c * nc + i] = 1.0;
    }
}

// Column (c, i) of the matrix for every probed cell c, from y = A e: row
// (c', i') of y belongs to the probed cell among c' and its face neighbours
// (at most one), and goes to the slab block of (slab of c', slab of c).
__global__ void k_probe_scatter(int dim, int m0, int m1, int m2, int nc, int64_t ndofs, int col0, int col1, int col2,
                                int i, const double *__restrict__ y, SlabBlocks blk) {
    const int mm[3] = {m0, m1, dim == 3 ? m2 : 1};
    const int col[3] = {col0, col1, col2};
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < ndofs;
         row += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cr = row / nc;
        const int ir = (int)(row - cr * nc);
        int c[3];
        c[0] = (int)(cr % m0);
        const int64_t r0 = cr / m0;
        c[1] = dim == 3 ? (int)(r0 % m1) : (int)r0;
        c[2] = dim == 3 ? (int)(r0 / m1) : 0;
        for (int o = 0; o <= 2 * dim; ++o) {  // o = 0: the cell itself, then -e_a, +e_a
            int p[3] = {c[0], c[1], c[2]};
            if (o > 0) p[(o - 1) / 2] += (o % 2) ? -1 : 1;
            bool ok = true;
            for (int a = 0; a < dim; ++a) ok = ok && p[a] >= 0 && p[a] < mm[a] && p[a] % 3 == col[a];
            if (!ok) continue;
            const int s_row = c[dim - 1], s_col = p[dim - 1];
            const int64_t in_row = dim == 3 ? c[0] + (int64_t)m0 * c[1] : c[0];
            const int64_t in_col = dim == 3 ? p[0] + (int64_t)m0 * p[1] : p[0];
            const int64_t B = blk.B;
            double *base = s_col == s_row ? blk.D + s_row * B * B
                                          : (s_col == s_row - 1 ? blk.Lo + (s_row - 1) * B * B : blk.Up + s_row * B * B);
            base[(in_row * nc + ir) + (in_col * nc + i) * B] = y[row];
            break;
        }
    }
}

}  // namespace fts

struct fts_mapped_hierarchy {
    int nlevels = 0, m_pre = 1, m_post = 1;
    int smoother = FTS_SMOOTHER_ADDITIVE;
    int local = FTS_LOCAL_SURROGATE;
    std::vector<double> omega;
    std::vector<fts_mapped_level *> levels;  // 0 = coarsest
    std::vector<fts_level *> shapes;  // Cartesian levels of the same cell counts and degree (transfers, slab shape)
    std::vector<double *> vb, vx, vr;
    std::vector<double *> inv;  // per level >= 1 (built on request): inverses of the cell blocks R_K A R_K^T
    fts::CoarseLU *coarse = nullptr;
    double *host_scalars = nullptr;
};

namespace fts {

// Exact cell solvers on mapped meshes: the diagonal blocks A_KK = R_K A R_K^T
// of the mapped operator, probed with the red-black coloring (a cell's face
// neighbours all have the other color, so (A e)|_K = A_KK e_K when e is zero
// on every cell of the other color) and inverted in LDS.

// e[(c, i)] = 1 on the cells c of `color`, 0 elsewhere.
__global__ void k_cell_probe_set(int dim, int m0, int m1, int64_t ncells, int nc, int color, int i,
                                 double *__restrict__ e) {
    const int64_t n = ncells * nc;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / nc;
        e[q] = (q - c * nc == i && cell_parity(dim, m0, m1, c) == color) ? 1.0 : 0.0;
    }
}

// blk[c][row][i] = y[c nc + row] on the cells c of `color`.
__global__ void k_cell_probe_take(int dim, int m0, int m1, int64_t ncells, int nc, int color, int i,
                                  const double *__restrict__ y, double *__restrict__ blk) {
    const int64_t n = ncells * nc;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / nc;
        if (cell_parity(dim, m0, m1, c) != color) continue;
        const int row = (int)(q - c * nc);
        blk[(c * nc + row) * nc + i] = y[q];
    }
}

// In-place Gauss-Jordan inversion of one nc x nc block per workgroup, in LDS
// (no pivoting: the blocks are symmetric positive definite).
__global__ void __launch_bounds__(256) k_invert_cells(int nc, double *__restrict__ blk) {
    extern __shared__ double lds[];
    double *a = lds, *col = lds + nc * nc;
    double *g = blk + (int64_t)blockIdx.x * nc * nc;
    const int t = threadIdx.x, nn = nc * nc;
    for (int q = t; q < nn; q += blockDim.x) a[q] = g[q];
    for (int p = 0; p < nc; ++p) {
        __syncthreads();
        for (int i = t; i < nc; i += blockDim.x) col[i] = a[i * nc + p];
        __syncthreads();
        const double piv = col[p];
        for (int j = t; j < nc; j += blockDim.x) a[p * nc + j] = (j == p ? 1.0 : a[p * nc + j]) / piv;
        __syncthreads();
        for (int q = t; q < nn; q += blockDim.x) {
            const int i = q / nc, j = q - i * nc;
            if (i != p) a[q] = (j == p ? 0.0 : a[q]) - col[i] * a[p * nc + j];
        }
    }
    __syncthreads();
    for (int q = t; q < nn; q += blockDim.x) g[q] = a[q];
}

// x += omega A_KK^-1 r_K on the cells of `color` (every cell if color < 0);
// one workgroup per cell, one thread per row (A_KK^-1 is symmetric, so row
// `row` is read as column `row`: coalesced across the threads).
__global__ void __launch_bounds__(64) k_mapped_exact(int dim, int m0, int m1, int nc, double omega, int color,
                                                     const double *__restrict__ inv, const double *__restrict__ r,
                                                     double *__restrict__ x) {
    extern __shared__ double rs[];
    const int64_t c = blockIdx.x;
    if (color >= 0 && cell_parity(dim, m0, m1, c) != color) return;  // uniform over the workgroup
    const double *ic = inv + c * nc * nc;
    for (int q = threadIdx.x; q < nc; q += blockDim.x) rs[q] = r[c * nc + q];
    __syncthreads();
    for (int row = threadIdx.x; row < nc; row += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < nc; ++j) acc = fma(ic[(int64_t)j * nc + row], rs[j], acc);
        x[c * nc + row] += omega * acc;
    }
}

constexpr int kExactMaxNc = 64;  // the inversion keeps a block and a column in LDS

static fts_status build_exact_inverses(const fts_mapped_level *lv, double **out) {
    *out = nullptr;
    const int nc = (int)(lv->ndofs / lv->ncells);
    if (nc > kExactMaxNc)
        return fail(FTS_E_UNSUPPORTED, "exact cell solvers on mapped meshes: at most 64 unknowns per cell");
    double *blk = nullptr, *e = nullptr, *y = nullptr;
    const int64_t N = lv->ndofs;
    fts_status st = FTS_OK;
    if (dev_malloc(&blk, (size_t)lv->ncells * nc * nc * sizeof(double)) != hipSuccess ||
        dev_malloc(&e, N * sizeof(double)) != hipSuccess || dev_malloc(&y, N * sizeof(double)) != hipSuccess)
        st = fail(FTS_E_HIP, "device allocation of the exact cell solvers failed");
    const unsigned grid = (unsigned)std::min<int64_t>((N + 255) / 256, 8192);
    for (int color = 0; color < 2 && st == FTS_OK; ++color)
        for (int i = 0; i < nc && st == FTS_OK; ++i) {
            k_cell_probe_set<<<grid, 256>>>(lv->dim, lv->m[0], lv->m[1], lv->ncells, nc, color, i, e);
            st = run_mapped(lv, 0, 0.0, e, nullptr, y, nullptr);
            if (st == FTS_OK) {
                k_cell_probe_take<<<grid, 256>>>(lv->dim, lv->m[0], lv->m[1], lv->ncells, nc, color, i, y, blk);
                const hipError_t he = hipGetLastError();
                if (he != hipSuccess) st = hip_fail(he, "cell probing");
            }
        }
    if (st == FTS_OK) {
        k_invert_cells<<<dim3((unsigned)lv->ncells), 256, (size_t)(nc * nc + nc) * sizeof(double)>>>(nc, blk);
        const hipError_t he = hipGetLastError();
        if (he != hipSuccess) st = hip_fail(he, "k_invert_cells launch");
    }
    if (st == FTS_OK && hipDeviceSynchronize() != hipSuccess) st = fail(FTS_E_HIP, "exact cell solver setup failed");
    dev_free(e);
    dev_free(y);
    if (st != FTS_OK) {
        dev_free(blk);
        return st;
    }
    *out = blk;
    return FTS_OK;
}

// x += omega sum_K (local solve of K) r_K over the cells of `color` (all if
// color < 0), with the hierarchy's local solvers on level l.
static fts_status local_apply(const fts_mapped_hierarchy *h, int l, const double *r, double *x, int color,
                              hipStream_t s) {
    const fts_mapped_level *lv = h->levels[l];
    if (h->local != FTS_LOCAL_EXACT) return run_mapped(lv, 2, h->omega[l], r, nullptr, x, s, color);
    if (lv->ncells == 0) return FTS_OK;
    const int nc = (int)(lv->ndofs / lv->ncells);
    k_mapped_exact<<<dim3((unsigned)lv->ncells), 64, nc * sizeof(double), s>>>(lv->dim, lv->m[0], lv->m[1], nc,
                                                                               h->omega[l], color, h->inv[l], r, x);
    const hipError_t he = hipGetLastError();
    return he == hipSuccess ? FTS_OK : hip_fail(he, "k_mapped_exact launch");
}

static fts_status mapped_vcycle_level(fts_mapped_hierarchy *h, int l, const double *b, double *x, hipStream_t s,
                                      bool x_zero) {
    if (l == 0) return coarse_solve(h->coarse, b, x, s);
    const fts_mapped_level *lv = h->levels[l];
    double *r = h->vr[l];
    fts_status st = FTS_OK;
    auto smooth = [&](bool first_zero, bool post) {
        // additive: r = b - A x (b itself when x = 0), x += omega sum_K
        // Atilde_K^-1 r_K; multiplicative: the same per red-black color with
        // the residual recomputed before each, black first after the coarse
        // correction (the reversed order keeps the V-cycle symmetric)
        if (h->smoother != FTS_SMOOTHER_MULTIPLICATIVE) {
            fts_status e = first_zero ? FTS_OK : run_mapped(lv, 1, 0.0, x, b, r, s);
            if (e == FTS_OK) e = local_apply(h, l, first_zero ? b : r, x, -1, s);
            return e;
        }
        fts_status e = FTS_OK;
        for (int ci = 0; ci < 2 && e == FTS_OK; ++ci) {
            const bool zero = first_zero && ci == 0;
            if (!zero) e = run_mapped(lv, 1, 0.0, x, b, r, s);
            if (e == FTS_OK) e = local_apply(h, l, zero ? b : r, x, post ? 1 - ci : ci, s);
        }
        return e;
    };
    for (int i = 0; i < h->m_pre && st == FTS_OK; ++i) st = smooth(x_zero && i == 0, false);
    if (st == FTS_OK) st = run_mapped(lv, 1, 0.0, x, b, r, s);
    if (st == FTS_OK) st = launch_restrict(h->shapes[l - 1], h->shapes[l], r, h->vb[l - 1], s);
    if (st == FTS_OK && l - 1 > 0) st = launch_fill(h->vx[l - 1], h->levels[l - 1]->ndofs, 0.0, s);
    if (st == FTS_OK) st = mapped_vcycle_level(h, l - 1, h->vb[l - 1], h->vx[l - 1], s, true);
    if (st == FTS_OK) st = launch_prolongate(h->shapes[l - 1], h->shapes[l], h->vx[l - 1], x, s);
    for (int i = 0; i < h->m_post && st == FTS_OK; ++i) st = smooth(false, true);
    return st;
}

static fts_status mapped_readback(fts_mapped_hierarchy *h, const double *dev, hipStream_t s, double *out2) {
    FTS_HIP_CHECK(hipMemcpyAsync(h->host_scalars, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    FTS_HIP_CHECK(hipStreamSynchronize(s));
    out2[0] = h->host_scalars[0];
    out2[1] = h->host_scalars[1];
    return FTS_OK;
}

}  // namespace fts

extern "C" {

fts_status fts_mapped_hierarchy_destroy(fts_mapped_hierarchy *h) {
    if (!h) return FTS_OK;
    if (h->coarse) coarse_destroy(h->coarse);
    for (auto *p : h->vb) dev_free(p);
    for (auto *p : h->vx) dev_free(p);
    for (auto *p : h->vr) dev_free(p);
    for (auto *p : h->inv) dev_free(p);
    for (auto *l : h->levels) fts_mapped_level_destroy(l);
    for (auto *l : h->shapes) fts_level_destroy(l);
    if (h->host_scalars) (void)hipHostFree(h->host_scalars);
    delete h;
    return FTS_OK;
}

fts_status fts_mapped_hierarchy_create(const fts_mapped_desc *levels, int32_t nlevels, const double *omega_per_level,
                                       int32_t m_pre, int32_t m_post, fts_mapped_hierarchy **out) {
    if (!levels || !omega_per_level || !out) return fail(FTS_E_INVAL, "fts_mapped_hierarchy_create: NULL argument");
    *out = nullptr;
    if (nlevels < 1 || nlevels > 16) return fail(FTS_E_INVAL, "nlevels must be in 1..16");
    if (m_pre < 0 || m_post < 0) return fail(FTS_E_INVAL, "negative smoothing step count");
    const int d = levels[0].dim;
    for (int l = 0; l < nlevels; ++l) {
        if (levels[l].dim != d || levels[l].degree != levels[0].degree)
            return fail(FTS_E_INVAL, "all levels need the same dimension and degree");
        for (int a = 0; a < d; ++a)
            if (l > 0 && levels[l].ncells[a] != 2 * levels[l - 1].ncells[a])
                return fail(FTS_E_INVAL, "each level must have twice the cells of the previous one per axis");
    }
    fts_mapped_hierarchy *h = new fts_mapped_hierarchy();
    h->nlevels = nlevels;
    h->m_pre = m_pre;
    h->m_post = m_post;
    h->omega.assign(omega_per_level, omega_per_level + nlevels);
    fts_status st = FTS_OK;
    for (int l = 0; l < nlevels && st == FTS_OK; ++l) {
        fts_mapped_level *lv = nullptr;
        st = fts_mapped_level_create(&levels[l], &lv);
        if (st != FTS_OK) break;
        h->levels.push_back(lv);
        std::vector<double> w[3];
        fts_mesh_desc cd{};
        cd.dim = d;
        cd.degree = levels[l].degree;
        cd.penalty_factor = 1.0;
        for (int a = 0; a < 3; ++a) {
            cd.ncells[a] = a < d ? levels[l].ncells[a] : 1;
            w[a].assign(cd.ncells[a], 1.0 / cd.ncells[a]);
            cd.h[a] = w[a].data();
        }
        fts_level *shape = nullptr;
        st = fts_level_create(&cd, &shape);
        if (st != FTS_OK) break;
        h->shapes.push_back(shape);
        double *pb = nullptr, *px = nullptr, *pr = nullptr;
        const size_t bytes = (size_t)lv->ndofs * sizeof(double);
        if (l < nlevels - 1 && (dev_malloc(&pb, bytes) != hipSuccess || dev_malloc(&px, bytes) != hipSuccess))
            st = fail(FTS_E_HIP, "device allocation of level vectors failed");
        if (st == FTS_OK && dev_malloc(&pr, bytes) != hipSuccess)
            st = fail(FTS_E_HIP, "device allocation of level vectors failed");
        h->vb.push_back(pb);
        h->vx.push_back(px);
        h->vr.push_back(pr);
    }
    if (st == FTS_OK) {
        // A_0 by probing: for each class of cells (indices modulo 3) and local
        // DoF i, y = A e with e = 1 at DoF i of every cell of the class
        const fts_mapped_level *l0 = h->levels[0];
        const int64_t N = l0->ndofs, nc = N / l0->ncells;
        double *e = nullptr, *y = nullptr;
        if (dev_malloc(&e, N * sizeof(double)) != hipSuccess || dev_malloc(&y, N * sizeof(double)) != hipSuccess)
            st = fail(FTS_E_HIP, "device allocation of the probing vectors failed");
        auto fill = [&](const SlabBlocks &blk) -> fts_status {
            const int ncls = d == 3 ? 27 : 9;
            const unsigned gc = (unsigned)std::min<int64_t>((l0->ncells + 255) / 256, 4096);
            const unsigned gr = (unsigned)std::min<int64_t>((N + 255) / 256, 4096);
            for (int cls = 0; cls < ncls; ++cls) {
                const int c0 = cls % 3, c1 = (cls / 3) % 3, c2 = cls / 9;
                for (int i = 0; i < nc; ++i) {
                    fts_status f = launch_fill(e, N, 0.0, nullptr);
                    if (f != FTS_OK) return f;
                    k_probe_set<<<gc, 256>>>(d, l0->m[0], l0->m[1], l0->ncells, (int)nc, c0, c1, c2, i, e);
                    f = run_mapped(l0, 0, 0.0, e, nullptr, y, nullptr);
                    if (f != FTS_OK) return f;
                    k_probe_scatter<<<gr, 256>>>(d, l0->m[0], l0->m[1], l0->m[2], (int)nc, N, c0, c1, c2, i, y, blk);
                    const hipError_t he = hipGetLastError();
                    if (he != hipSuccess) return hip_fail(he, "coarse probing");
                }
            }
            return FTS_OK;
        };
        if (st == FTS_OK) st = coarse_create_with(h->shapes[0], fill, nullptr, &h->coarse);
        dev_free(e);
        dev_free(y);
        if (st == FTS_OK && hipHostMalloc(&h->host_scalars, 4 * sizeof(double)) != hipSuccess)
            st = fail(FTS_E_HIP, "hipHostMalloc of the readback buffer failed");
    }
    if (st != FTS_OK) {
        fts_mapped_hierarchy_destroy(h);
        return st;
    }
    *out = h;
    return FTS_OK;
}

int64_t fts_mapped_hierarchy_ndofs(const fts_mapped_hierarchy *h) { return h ? h->levels.back()->ndofs : -1; }

fts_status fts_mapped_hierarchy_set_local_solver(fts_mapped_hierarchy *h, int32_t local) {
    if (!h) return fail(FTS_E_INVAL, "fts_mapped_hierarchy_set_local_solver: NULL hierarchy");
    if (local != FTS_LOCAL_SURROGATE && local != FTS_LOCAL_EXACT)
        return fail(FTS_E_INVAL, "fts_mapped_hierarchy_set_local_solver: unknown local solver");
    if (local == FTS_LOCAL_EXACT) {
        h->inv.resize(h->nlevels, nullptr);
        for (int l = 1; l < h->nlevels; ++l) {
            if (h->inv[l]) continue;
            fts_status st = build_exact_inverses(h->levels[l], &h->inv[l]);
            if (st != FTS_OK) return st;
        }
    }
    h->local = local;
    return FTS_OK;
}

fts_status fts_mapped_hierarchy_set_smoother(fts_mapped_hierarchy *h, int32_t smoother) {
    if (!h) return fail(FTS_E_INVAL, "fts_mapped_hierarchy_set_smoother: NULL hierarchy");
    if (smoother != FTS_SMOOTHER_ADDITIVE && smoother != FTS_SMOOTHER_MULTIPLICATIVE)
        return fail(FTS_E_INVAL, "fts_mapped_hierarchy_set_smoother: unknown smoother");
    h->smoother = smoother;
    return FTS_OK;
}

fts_status fts_mapped_vcycle(fts_mapped_hierarchy *h, const double *b, double *x, void *stream) {
    if (!h || !b || !x) return fail(FTS_E_INVAL, "fts_mapped_vcycle: NULL argument");
    return mapped_vcycle_level(h, h->nlevels - 1, b, x, reinterpret_cast<hipStream_t>(stream), false);
}

size_t fts_mapped_pcg_ws_bytes(const fts_mapped_hierarchy *h) {
    if (!h) return 0;
    return (size_t)(5 * h->levels.back()->ndofs + 2 * red_partials() + 2) * sizeof(double);
}

fts_status fts_mapped_pcg(fts_mapped_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit, void *ws,
                          size_t ws_bytes, int32_t *iters, double *relres, double *history, void *stream) {
    if (!h || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_mapped_pcg: NULL argument");
    if (ws_bytes < fts_mapped_pcg_ws_bytes(h)) return fail(FTS_E_SIZE, "fts_mapped_pcg: workspace too small");
    if (!(rtol >= 0.0) || maxit < 0) return fail(FTS_E_INVAL, "fts_mapped_pcg: invalid rtol or maxit");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const fts_mapped_level *lv = h->levels.back();
    const int64_t N = lv->ndofs;
    double *r = static_cast<double *>(ws), *z = r + N, *zo = z + N, *p = zo + N, *q = p + N;
    double *part = q + N, *dout = part + 2 * red_partials();
    double v[2];
    fts_status st;
#define FTS_TRY(expr)                    \
    do {                                 \
        st = (expr);                     \
        if (st != FTS_OK) return st;     \
    } while (0)
    FTS_TRY(run_mapped(lv, 1, 0.0, x, b, r, s));
    FTS_TRY(launch_dot2(b, b, nullptr, N, part, dout, s));
    FTS_TRY(mapped_readback(h, dout, s, v));
    const double bb = v[0];
    FTS_TRY(launch_dot2(r, r, nullptr, N, part, dout, s));
    FTS_TRY(mapped_readback(h, dout, s, v));
    double rel = bb > 0.0 ? std::sqrt(v[0] / bb) : 0.0;
    if (history) history[0] = rel;
    int it = 0;
    if (rel > rtol && maxit > 0) {
        FTS_TRY(launch_fill(z, N, 0.0, s));
        FTS_TRY(mapped_vcycle_level(h, h->nlevels - 1, r, z, s, true));
        FTS_HIP_CHECK(hipMemcpyAsync(p, z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        FTS_TRY(launch_dot2(r, z, nullptr, N, part, dout, s));
        FTS_TRY(mapped_readback(h, dout, s, v));
        double rz = v[0];
        while (it < maxit) {
            FTS_TRY(run_mapped(lv, 0, 0.0, p, nullptr, q, s));
            FTS_TRY(launch_dot2(p, q, nullptr, N, part, dout, s));
            FTS_TRY(mapped_readback(h, dout, s, v));
            const double alpha = rz / v[0];
            FTS_TRY(launch_cg_update(x, r, p, q, alpha, N, s));
            FTS_TRY(launch_dot2(r, r, nullptr, N, part, dout, s));
            FTS_TRY(mapped_readback(h, dout, s, v));
            rel = std::sqrt(v[0] / bb);
            ++it;
            if (history) history[it] = rel;
            if (!(rel > rtol)) break;
            std::swap(z, zo);
            FTS_TRY(launch_fill(z, N, 0.0, s));
            FTS_TRY(mapped_vcycle_level(h, h->nlevels - 1, r, z, s, true));
            FTS_TRY(launch_dot2(r, z, zo, N, part, dout, s));
            FTS_TRY(mapped_readback(h, dout, s, v));
            // flexible (Polak-Ribiere) update: beta = r.(z - z_old) / rz_old
            const double beta = (v[0] - v[1]) / rz;
            rz = v[0];
            FTS_TRY(launch_xpby(p, z, beta, N, s));
        }
    }
#undef FTS_TRY
    if (iters) *iters = it;
    if (relres) *relres = rel;
    return FTS_OK;
}

}  // extern "C"
