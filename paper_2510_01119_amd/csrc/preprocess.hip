// Per-(view, Gaussian) slice + project, forward and backward.
//
// Forward (Sec. 3.3 Eq. "4dgs"; Sec. 3.3 "Motion-Aware Gaussian"; Sec. 3.1):
//   activations -> 4D rotation from the left/right quaternion pair ->
//   Sigma = (R S)(R S)^T -> conditional 3D Gaussian at time t and temporal
//   opacity o_t -> temporal / near / determinant culls -> EWA projection
//   (guard-banded Jacobian, 0.3 px^2 dilation) -> conic, mean2D -> exact
//   alpha >= 1/255 footprint -> 16x16 tile rectangle.
//
// Every value here that decides an integer (cull, rectangle, the depth bits
// of the sort key) must be reproducible bit for bit, so this file is compiled
// without floating-point contraction, sums run left to right, divisions and
// square roots are the correctly rounded IEEE operations, and exp / ln are
// the two project-defined FP32 routines below.  One thread handles one
// (view, Gaussian); parameters are read as coalesced SoA planes.
#include <cmath>

#include "common.hpp"

#pragma clang fp contract(off)

namespace gs4d {
namespace {

// Everything the backward needs from the forward of one (view, Gaussian).
struct Slice {
    float s[4], o;
    float nl, nr, ql[4], qr[4];
    float A[4][4], B[4][4];   // left / right multiplication matrices
    float R[4][4];            // rotation in (x, y, z, t) order
    float M[4][4];            // R diag(s)
    float Sg[4][4];           // 4D covariance
    float P[3][4];            // rows of M with the time direction projected out
    float dt, ef, ot;         // t - mu_t, exp(-dt^2 / 2c), o_t
    float mu[3], Sc[3][3];    // conditional mean / covariance
    float xc[3];              // camera-space point
    float ux, uy;             // guard-banded x/z, y/z
    int clx, cly;             // guard band active
    float J00, J02, J11, J12;
    float T[2][3], U[2][3];   // T = J W, U = T Sc
    float sa, sb, sc, det;    // Sigma2D = [[sa, sb], [sb, sc]]
    float ca, cb, cc;         // conic
    float mx, my;
    float hx, hy;             // footprint half-widths
};

__device__ __forceinline__ int project_slice(const gs4d_view &V, Slice &S, int4 *rect_out);

// Returns 1 if the Gaussian is visible; `touched`/`rect` filled when asked.
__device__ __forceinline__ int slice_project(const float (&p)[20], const gs4d_view &V, Slice &S,
                                             int4 *rect_out) {
    for (int k = 0; k < 20; ++k)
        if (!isfinite(p[k])) return 0;

    for (int k = 0; k < 4; ++k) S.s[k] = fixed_exp(p[4 + k]);
    S.o = 1.0f / (1.0f + fixed_exp(-p[16]));

    S.nl = sqrtf(p[8] * p[8] + p[9] * p[9] + p[10] * p[10] + p[11] * p[11]);
    S.nr = sqrtf(p[12] * p[12] + p[13] * p[13] + p[14] * p[14] + p[15] * p[15]);
    if (!(S.nl > 0.0f) || !(S.nr > 0.0f)) return 0;
    for (int k = 0; k < 4; ++k) {
        S.ql[k] = p[8 + k] / S.nl;
        S.qr[k] = p[12 + k] / S.nr;
    }
    const float *a = S.ql, *b = S.qr;
    // left multiplication by a, right multiplication by b, basis (1, i, j, k)
    const float Am[4][4] = {{a[0], -a[1], -a[2], -a[3]},
                            {a[1], a[0], -a[3], a[2]},
                            {a[2], a[3], a[0], -a[1]},
                            {a[3], -a[2], a[1], a[0]}};
    const float Bm[4][4] = {{b[0], -b[1], -b[2], -b[3]},
                            {b[1], b[0], b[3], -b[2]},
                            {b[2], -b[3], b[0], b[1]},
                            {b[3], b[2], -b[1], b[0]}};
    float Q[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            S.A[i][j] = Am[i][j];
            S.B[i][j] = Bm[i][j];
            Q[i][j] = Am[i][0] * Bm[0][j] + Am[i][1] * Bm[1][j] + Am[i][2] * Bm[2][j] +
                      Am[i][3] * Bm[3][j];
        }
    // (x, y, z, t) <- quaternion axes (i, j, k, 1)
    const int perm[4] = {1, 2, 3, 0};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            S.R[i][j] = Q[perm[i]][perm[j]];
            S.M[i][j] = S.R[i][j] * S.s[j];
        }
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) {
            const float v = S.M[i][0] * S.M[j][0] + S.M[i][1] * S.M[j][1] +
                            S.M[i][2] * S.M[j][2] + S.M[i][3] * S.M[j][3];
            S.Sg[i][j] = v;
            S.Sg[j][i] = v;
        }
    const float c = S.Sg[3][3];
    if (!(c > 0.0f)) return 0;

    // conditional at time t.  With m = M[3] (the time row), c = m.m and
    // a_i = M_i.m = Sg[i][3], the conditional covariance Sg_xyz - a a^T / c
    // equals P P^T with P_i = M_i - (a_i / c) m: each row with the time
    // direction projected out.  That form keeps FP32 accuracy when
    // s_t >> s_xyz, where the difference of the two blocks would cancel
    // (an error of order eps (s_t / s_xyz)^2 relative to Sc).
    S.dt = V.t - p[3];
    const float r = S.dt / c;
    for (int i = 0; i < 3; ++i) S.mu[i] = p[i] + S.Sg[i][3] * r;
    for (int i = 0; i < 3; ++i) {
        const float k = S.Sg[i][3] / c;
        for (int j = 0; j < 4; ++j) S.P[i][j] = S.M[i][j] - k * S.M[3][j];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const float v = S.P[i][0] * S.P[j][0] + S.P[i][1] * S.P[j][1] +
                            S.P[i][2] * S.P[j][2] + S.P[i][3] * S.P[j][3];
            S.Sc[i][j] = v;
            S.Sc[j][i] = v;
        }
    const float qd = (S.dt * S.dt) / c;
    S.ef = fixed_exp(-0.5f * qd);
    S.ot = S.o * S.ef;
    return project_slice(V, S, rect_out);
}

// Isotropic, motion-aware parameters (13 per Gaussian: mean xyz t, log s,
// log s_t, velocity v, opacity logit, rgb), Sec. 3.3: the 4D covariance
// [[s^2 I + s_t^2 v v^T, s_t^2 v], [s_t^2 v^T, s_t^2]] has, at time t, the
// conditional mean mu + v (t - mu_t), covariance s^2 I and o_t = o exp(-(t -
// mu_t)^2 / (2 s_t^2)).  S.s[0] = s, S.s[3] = s_t.
__device__ __forceinline__ int slice_project_iso(const float (&p)[GS4D_ISO_FIELDS],
                                                 const gs4d_view &V, Slice &S, int4 *rect_out) {
    for (int k = 0; k < GS4D_ISO_FIELDS; ++k)
        if (!isfinite(p[k])) return 0;
    S.s[0] = fixed_exp(p[4]);
    S.s[3] = fixed_exp(p[5]);
    S.o = 1.0f / (1.0f + fixed_exp(-p[9]));
    const float c = S.s[3] * S.s[3];
    if (!(c > 0.0f)) return 0;
    S.dt = V.t - p[3];
    for (int i = 0; i < 3; ++i) S.mu[i] = p[i] + p[6 + i] * S.dt;
    const float s2 = S.s[0] * S.s[0];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S.Sc[i][j] = i == j ? s2 : 0.0f;
    const float qd = (S.dt * S.dt) / c;
    S.ef = fixed_exp(-0.5f * qd);
    S.ot = S.o * S.ef;
    return project_slice(V, S, rect_out);
}

// ---------------------------------------------------------------- projection
// From the conditional 3D Gaussian (S.mu, S.Sc, S.ot) to the record: the
// temporal cull, camera space, the guard-banded EWA Jacobian, Sigma2D and
// its conic, the exact footprint and its tile rectangle.
__device__ __forceinline__ int project_slice(const gs4d_view &V, Slice &S, int4 *rect_out) {
    if (!(255.0f * S.ot >= 1.0f)) return 0;

    // camera space
    const float *Rt = V.Rt;
    for (int i = 0; i < 3; ++i)
        S.xc[i] = Rt[4 * i] * S.mu[0] + Rt[4 * i + 1] * S.mu[1] + Rt[4 * i + 2] * S.mu[2] +
                  Rt[4 * i + 3];
    const float z = S.xc[2];
    if (!(z >= V.near_z)) return 0;

    // EWA Jacobian at the guard-banded direction
    const float limx = 1.3f * ((0.5f * (float)V.width) / V.fx);
    const float limy = 1.3f * ((0.5f * (float)V.height) / V.fy);
    const float ux0 = S.xc[0] / z, uy0 = S.xc[1] / z;
    S.ux = fminf(fmaxf(ux0, -limx), limx);
    S.uy = fminf(fmaxf(uy0, -limy), limy);
    S.clx = (ux0 < -limx) || (ux0 > limx);
    S.cly = (uy0 < -limy) || (uy0 > limy);
    S.J00 = V.fx / z;
    S.J02 = -(V.fx * S.ux) / z;
    S.J11 = V.fy / z;
    S.J12 = -(V.fy * S.uy) / z;
    for (int j = 0; j < 3; ++j) {
        S.T[0][j] = S.J00 * Rt[j] + S.J02 * Rt[8 + j];
        S.T[1][j] = S.J11 * Rt[4 + j] + S.J12 * Rt[8 + j];
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            S.U[i][j] = S.T[i][0] * S.Sc[0][j] + S.T[i][1] * S.Sc[1][j] + S.T[i][2] * S.Sc[2][j];
    S.sa = S.U[0][0] * S.T[0][0] + S.U[0][1] * S.T[0][1] + S.U[0][2] * S.T[0][2] + 0.3f;
    S.sb = S.U[0][0] * S.T[1][0] + S.U[0][1] * S.T[1][1] + S.U[0][2] * S.T[1][2];
    S.sc = S.U[1][0] * S.T[1][0] + S.U[1][1] * S.T[1][1] + S.U[1][2] * S.T[1][2] + 0.3f;
    S.det = S.sa * S.sc - S.sb * S.sb;
    if (!(S.det > 0.0f)) return 0;
    S.ca = S.sc / S.det;
    S.cb = -S.sb / S.det;
    S.cc = S.sa / S.det;
    S.mx = V.fx * ux0 + V.cx;
    S.my = V.fy * uy0 + V.cy;

    // exact footprint: alpha >= 1/255 iff d^T conic d <= 2 ln(255 o_t)
    const float tau = 2.0f * fixed_log(255.0f * S.ot);
    const float taub = tau * 1.0009765625f + 0.0009765625f;
    const float hx = sqrtf(taub * S.sa), hy = sqrtf(taub * S.sc);
    if (!isfinite(S.mx) || !isfinite(S.my) || !isfinite(hx) || !isfinite(hy) ||
        !isfinite(S.ca) || !isfinite(S.cb) || !isfinite(S.cc))
        return 0;
    float x0 = ceilf((S.mx - hx) - 0.5f), x1 = floorf((S.mx + hx) - 0.5f);
    float y0 = ceilf((S.my - hy) - 0.5f), y1 = floorf((S.my + hy) - 0.5f);
    x0 = fminf(fmaxf(x0, 0.0f), (float)V.width);
    y0 = fminf(fmaxf(y0, 0.0f), (float)V.height);
    x1 = fmaxf(fminf(x1, (float)(V.width - 1)), -1.0f);
    y1 = fmaxf(fminf(y1, (float)(V.height - 1)), -1.0f);
    const int px0 = (int)x0, px1 = (int)x1, py0 = (int)y0, py1 = (int)y1;
    if (px0 > px1 || py0 > py1) return 0;
    if (rect_out) *rect_out = make_int4(px0 >> 4, py0 >> 4, (px1 >> 4) + 1, (py1 >> 4) + 1);
    S.hx = hx;
    S.hy = hy;
    return 1;
}

__global__ void __launch_bounds__(256)
preprocess_fwd_kernel(const float *__restrict__ P, int64_t n, ViewPack vp, float4 *__restrict__ rec,
                      int4 *__restrict__ rect, int32_t *__restrict__ touched) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int vi = blockIdx.y;
    if (g >= n) return;
    float p[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) p[k] = P[(int64_t)k * n + g];
    Slice S;
    int4 rc = make_int4(0, 0, 0, 0);
    const int vis = slice_project(p, vp.v[vi], S, &rc);
    const int64_t o = (int64_t)vi * n + g;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    int tt = 0;
    if (vis) {
        r0 = make_float4(S.mx, S.my, S.ca, S.cb);
        r1 = make_float4(S.cc, S.ot, S.xc[2], S.hx);
        r2 = make_float4(p[17], p[18], p[19], S.hy);
        tt = (rc.z - rc.x) * (rc.w - rc.y);
    } else {
        rc = make_int4(0, 0, 0, 0);
    }
    rec[3 * o + 0] = r0;
    rec[3 * o + 1] = r1;
    rec[3 * o + 2] = r2;
    rect[o] = rc;
    touched[o] = tt;
}

// Backward of project_slice for one record: d(mean2D, conic) -> d(conditional
// mean) Gmu and d(conditional covariance) GSc (chain rule term by term: conic
// -> Sigma2D (dS = -Q dQ Q), Sigma2D -> (T, Sc), T = J W -> J -> camera point,
// no gradient through a clamped guard-band coordinate).
__device__ __forceinline__ void project_bwd(const gs4d_view &V, const Slice &S, const float (&G)[9],
                                            float (&Gmu)[3], float (&GSc)[3][3]) {
    const float *Rt = V.Rt;
    const float z = S.xc[2];
    // conic -> Sigma2D:  G_S = -Q Gq Q, Gq = [[ga, gb/2], [gb/2, gc]]
    const float q00 = S.ca, q01 = S.cb, q11 = S.cc;
    const float g00 = G[2], g01 = 0.5f * G[3], g11 = G[4];
    const float t00 = g00 * q00 + g01 * q01, t01 = g00 * q01 + g01 * q11;
    const float t10 = g01 * q00 + g11 * q01, t11 = g01 * q01 + g11 * q11;
    const float S00 = -(q00 * t00 + q01 * t10);
    const float S01 = -(q00 * t01 + q01 * t11);
    const float S11 = -(q01 * t01 + q11 * t11);
    const float GS2[2][2] = {{S00, S01}, {S01, S11}};

    // Sigma2D = T Sc T^T: dSc = T^T GS2 T; dT = 2 GS2 U  (U = T Sc)
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            float accv = 0.0f;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) accv += S.T[k][i] * GS2[k][l] * S.T[l][j];
            GSc[i][j] = accv;
        }
    float GT[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            GT[i][j] = 2.0f * (GS2[i][0] * S.U[0][j] + GS2[i][1] * S.U[1][j]);
    // T = J W: dJ = dT W^T (only the non-constant entries of J)
    const float GJ00 = GT[0][0] * Rt[0] + GT[0][1] * Rt[1] + GT[0][2] * Rt[2];
    const float GJ02 = GT[0][0] * Rt[8] + GT[0][1] * Rt[9] + GT[0][2] * Rt[10];
    const float GJ11 = GT[1][0] * Rt[4] + GT[1][1] * Rt[5] + GT[1][2] * Rt[6];
    const float GJ12 = GT[1][0] * Rt[8] + GT[1][1] * Rt[9] + GT[1][2] * Rt[10];
    const float iz = 1.0f / z, iz2 = iz * iz;
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    gz += -(GJ00 * V.fx + GJ11 * V.fy) * iz2;
    if (S.clx) {
        gz += GJ02 * V.fx * S.ux * iz2;
    } else {
        gx += -GJ02 * V.fx * iz2;
        gz += GJ02 * 2.0f * V.fx * S.xc[0] * iz2 * iz;
    }
    if (S.cly) {
        gz += GJ12 * V.fy * S.uy * iz2;
    } else {
        gy += -GJ12 * V.fy * iz2;
        gz += GJ12 * 2.0f * V.fy * S.xc[1] * iz2 * iz;
    }
    // mean2D = (fx x/z + cx, fy y/z + cy)
    gx += G[0] * V.fx * iz;
    gy += G[1] * V.fy * iz;
    gz += -(G[0] * V.fx * S.xc[0] + G[1] * V.fy * S.xc[1]) * iz2;
    // camera point -> conditional mean
    for (int j = 0; j < 3; ++j) Gmu[j] = Rt[j] * gx + Rt[4 + j] * gy + Rt[8 + j] * gz;
}

// Chain rule of one (view, Gaussian) of the rotor form from the gradients of
// its conditional mean (Gmu), conditional covariance (GSc) and temporal
// opacity (go) to the raw parameters 0-16 (mean, log scales, both
// quaternions, opacity logit), added to acc.
__device__ __forceinline__ void rotor_chain(const Slice &S, const float (&Gmu)[3],
                                            const float (&GSc)[3][3], const float go,
                                            float (&acc)[20]) {
    // conditional -> (M, mu_t, opacity).  With K = [I | -a/c] the
    // covariance part of the Sigma gradient is K^T GSc K, and since
    // K M = P, its share of dL/dM = 2 G4 M is 2 K^T GSc P: rows 0-2 are
    // 2 GSc P, row 3 is -2 (a/c)^T GSc P (no cancelling terms when
    // s_t >> s_xyz).  The conditional mean and o_t add
    // G4_mo = [[0, g/2], [g^T/2, h]] with g = Gmu dt / c and
    // h = -(Gmu.a) dt / c^2 + go o_t dt^2 / (2 c^2).
    const float c = S.Sg[3][3], ic = 1.0f / c;
    const float dt = S.dt;
    float Gmua = 0.0f;
    for (int i = 0; i < 3; ++i) Gmua += Gmu[i] * S.Sg[i][3];
    for (int i = 0; i < 3; ++i) acc[i] += Gmu[i];
    acc[3] += -Gmua * ic + go * S.ot * dt * ic;
    const float Gdo = go * S.ef;
    float gv[3], kv[3];
    for (int i = 0; i < 3; ++i) {
        gv[i] = Gmu[i] * dt * ic;
        kv[i] = S.Sg[i][3] * ic;
    }
    const float h = (-Gmua * dt + 0.5f * go * S.ot * dt * dt) * ic * ic;
    float GM[4][4];
    for (int j = 0; j < 4; ++j) {
        float GP[3];
        for (int i = 0; i < 3; ++i)
            GP[i] = GSc[i][0] * S.P[0][j] + GSc[i][1] * S.P[1][j] + GSc[i][2] * S.P[2][j];
        for (int i = 0; i < 3; ++i) GM[i][j] = 2.0f * GP[i] + gv[i] * S.M[3][j];
        GM[3][j] = -2.0f * (kv[0] * GP[0] + kv[1] * GP[1] + kv[2] * GP[2]) +
                   (gv[0] * S.M[0][j] + gv[1] * S.M[1][j] + gv[2] * S.M[2][j]) +
                   2.0f * h * S.M[3][j];
    }
    float GR[4][4], Gs[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            GR[i][j] = GM[i][j] * S.s[j];
            Gs[j] += GM[i][j] * S.R[i][j];
        }
    // R = Pi (A B) Pi^T
    const int perm[4] = {1, 2, 3, 0};
    float GQ[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) GQ[perm[i]][perm[j]] = GR[i][j];
    float GA[4][4], GB[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            GA[i][j] = GQ[i][0] * S.B[j][0] + GQ[i][1] * S.B[j][1] + GQ[i][2] * S.B[j][2] +
                       GQ[i][3] * S.B[j][3];
            GB[i][j] = S.A[0][i] * GQ[0][j] + S.A[1][i] * GQ[1][j] + S.A[2][i] * GQ[2][j] +
                       S.A[3][i] * GQ[3][j];
        }
    // each matrix entry is +- one quaternion component
    float gl[4], gr[4];
    gl[0] = GA[0][0] + GA[1][1] + GA[2][2] + GA[3][3];
    gl[1] = -GA[0][1] + GA[1][0] - GA[2][3] + GA[3][2];
    gl[2] = -GA[0][2] + GA[1][3] + GA[2][0] - GA[3][1];
    gl[3] = -GA[0][3] - GA[1][2] + GA[2][1] + GA[3][0];
    gr[0] = GB[0][0] + GB[1][1] + GB[2][2] + GB[3][3];
    gr[1] = -GB[0][1] + GB[1][0] + GB[2][3] - GB[3][2];
    gr[2] = -GB[0][2] - GB[1][3] + GB[2][0] + GB[3][1];
    gr[3] = -GB[0][3] + GB[1][2] - GB[2][1] + GB[3][0];
    float dl = 0.0f, dr = 0.0f;
    for (int k = 0; k < 4; ++k) {
        dl += S.ql[k] * gl[k];
        dr += S.qr[k] * gr[k];
    }
    const float inl = 1.0f / S.nl, inr = 1.0f / S.nr;
    for (int k = 0; k < 4; ++k) {
        acc[4 + k] += Gs[k] * S.s[k];
        acc[8 + k] += (gl[k] - S.ql[k] * dl) * inl;
        acc[12 + k] += (gr[k] - S.qr[k] * dr) * inr;
    }
    acc[16] += Gdo * S.o * (1.0f - S.o);
}

// Backward: d(mean2D, conic, o_t, rgb) per (view, Gaussian) -> d(raw params),
// summed over views.  Follows the forward above term by term (chain rule):
// conic -> Sigma2D (dS = -Q dQ Q), Sigma2D -> (T, Sc), T = J W -> J -> camera
// point (no gradient through a clamped guard-band coordinate), camera ->
// conditional mean, conditional -> (Sigma blocks, mu_t, opacity), Sigma =
// M M^T -> (R, s), R -> (left, right) unit quaternions -> raw quaternions.
__global__ void __launch_bounds__(128, 3)
preprocess_bwd_kernel(const float *__restrict__ P, int64_t n, ViewPack vp,
                      const int32_t *__restrict__ touched, const float *__restrict__ grad2d,
                      float *__restrict__ dP) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float p[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) p[k] = P[(int64_t)k * n + g];
    float acc[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) acc[k] = 0.0f;

    for (int vi = 0; vi < vp.n_views; ++vi) {
        const int64_t o = (int64_t)vi * n + g;
        if (touched[o] == 0) continue;
        const gs4d_view &V = vp.v[vi];
        Slice S;
        if (!slice_project(p, V, S, nullptr)) continue;
        float G[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = grad2d[o * 9 + k];
        float Gmu[3], GSc[3][3];
        project_bwd(V, S, G, Gmu, GSc);

        rotor_chain(S, Gmu, GSc, G[5], acc);
        acc[17] += G[6];
        acc[18] += G[7];
        acc[19] += G[8];
    }
#pragma unroll
    for (int k = 0; k < 20; ++k) dP[(int64_t)k * n + g] = acc[k];
}

// Forward of the isotropic, motion-aware parameters [13][n]; the records,
// rectangles and counts have the layout of preprocess_fwd_kernel's.
__global__ void __launch_bounds__(256)
preprocess_iso_fwd_kernel(const float *__restrict__ P, int64_t n, ViewPack vp,
                          float4 *__restrict__ rec, int4 *__restrict__ rect,
                          int32_t *__restrict__ touched) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int vi = blockIdx.y;
    if (g >= n) return;
    float p[GS4D_ISO_FIELDS];
#pragma unroll
    for (int k = 0; k < GS4D_ISO_FIELDS; ++k) p[k] = P[(int64_t)k * n + g];
    Slice S;
    int4 rc = make_int4(0, 0, 0, 0);
    const int vis = slice_project_iso(p, vp.v[vi], S, &rc);
    const int64_t o = (int64_t)vi * n + g;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    int tt = 0;
    if (vis) {
        r0 = make_float4(S.mx, S.my, S.ca, S.cb);
        r1 = make_float4(S.cc, S.ot, S.xc[2], S.hx);
        r2 = make_float4(p[10], p[11], p[12], S.hy);
        tt = (rc.z - rc.x) * (rc.w - rc.y);
    } else {
        rc = make_int4(0, 0, 0, 0);
    }
    rec[3 * o + 0] = r0;
    rec[3 * o + 1] = r1;
    rec[3 * o + 2] = r2;
    rect[o] = rc;
    touched[o] = tt;
}

// Backward of the isotropic, motion-aware form, summed over views:
//   mu_c = mu + v dt (dt = t - mu_t): d mu += Gmu, d v += Gmu dt,
//     d mu_t -= v . Gmu;
//   Sc = s^2 I: d log s = 2 s^2 trace(GSc);
//   o_t = o exp(-dt^2 / (2 s_t^2)): d mu_t += go o_t dt / s_t^2,
//     d log s_t = go o_t dt^2 / s_t^2, d logit = go exp(.) o (1 - o).
__global__ void __launch_bounds__(128)
preprocess_iso_bwd_kernel(const float *__restrict__ P, int64_t n, ViewPack vp,
                          const int32_t *__restrict__ touched, const float *__restrict__ grad2d,
                          float *__restrict__ dP) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float p[GS4D_ISO_FIELDS];
#pragma unroll
    for (int k = 0; k < GS4D_ISO_FIELDS; ++k) p[k] = P[(int64_t)k * n + g];
    float acc[GS4D_ISO_FIELDS];
#pragma unroll
    for (int k = 0; k < GS4D_ISO_FIELDS; ++k) acc[k] = 0.0f;

    for (int vi = 0; vi < vp.n_views; ++vi) {
        const int64_t o = (int64_t)vi * n + g;
        if (touched[o] == 0) continue;
        const gs4d_view &V = vp.v[vi];
        Slice S;
        if (!slice_project_iso(p, V, S, nullptr)) continue;
        float G[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = grad2d[o * 9 + k];
        float Gmu[3], GSc[3][3];
        project_bwd(V, S, G, Gmu, GSc);
        const float go = G[5];
        const float ic = 1.0f / (S.s[3] * S.s[3]);
        const float dt = S.dt;
        float vG = 0.0f;
        for (int i = 0; i < 3; ++i) {
            acc[i] += Gmu[i];
            acc[6 + i] += Gmu[i] * dt;
            vG += p[6 + i] * Gmu[i];
        }
        acc[3] += -vG + go * S.ot * dt * ic;
        acc[4] += 2.0f * S.s[0] * S.s[0] * (GSc[0][0] + GSc[1][1] + GSc[2][2]);
        acc[5] += go * S.ot * dt * dt * ic;
        acc[9] += go * S.ef * S.o * (1.0f - S.o);
        acc[10] += G[6];
        acc[11] += G[7];
        acc[12] += G[8];
    }
#pragma unroll
    for (int k = 0; k < GS4D_ISO_FIELDS; ++k) dP[(int64_t)k * n + g] = acc[k];
}


// ---------------------------------------------------------------- SCH colour
// The sphericylindrical-harmonic appearance of 4D Gaussian splatting (Sec.
// 3.1, SCH equation): Z_{nl}^m(t, d) = cos(2 pi n t / T) Y_l^m(d) for
// degrees l <= L and temporal frequencies n <= N, d the unit direction from
// the camera centre to the conditional mean.  Y_l^m are the real spherical
// harmonics, orthonormal on the sphere, without the Condon-Shortley phase
// (Y_{1,1} = +c x, Y_{1,-1} = +c y), index l^2 + l + m, written as
// polynomials in (x, y, z); basis b = n (L+1)^2 + l^2 + l + m, coefficient
// row 3 b + channel.

// normalisation constants: sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), times sqrt(2)
// for m != 0, times the integer factor of each polynomial
#define SH_C0 0.28209479177387814f   // 1 / (2 sqrt(pi))
#define SH_C1 0.48860251190291992f   // sqrt(3 / (4 pi))
#define SH_C2A 1.0925484305920792f   // sqrt(15 / (4 pi))
#define SH_C2B 0.31539156525252005f  // sqrt(5 / (16 pi))
#define SH_C2C 0.54627421529603959f  // sqrt(15 / (16 pi))
#define SH_C3A 0.59004358992664352f  // sqrt(35 / (32 pi))
#define SH_C3B 2.8906114426405538f   // sqrt(105 / (4 pi))
#define SH_C3C 0.45704579946446572f  // sqrt(21 / (32 pi))
#define SH_C3D 0.37317633259011540f  // sqrt(7 / (16 pi))
#define SH_C3E 1.4453057213202769f   // sqrt(105 / (16 pi))

template <int L>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float (&Y)[(L + 1) * (L + 1)]) {
    Y[0] = SH_C0;
    if constexpr (L >= 1) {
        Y[1] = SH_C1 * y;
        Y[2] = SH_C1 * z;
        Y[3] = SH_C1 * x;
    }
    if constexpr (L >= 2) {
        Y[4] = SH_C2A * (x * y);
        Y[5] = SH_C2A * (y * z);
        Y[6] = SH_C2B * (3.0f * (z * z) - 1.0f);
        Y[7] = SH_C2A * (x * z);
        Y[8] = SH_C2C * (x * x - y * y);
    }
    if constexpr (L >= 3) {
        const float z5 = 5.0f * (z * z) - 1.0f;
        Y[9] = SH_C3A * (y * (3.0f * (x * x) - y * y));
        Y[10] = SH_C3B * (x * y * z);
        Y[11] = SH_C3C * (y * z5);
        Y[12] = SH_C3D * (z * (5.0f * (z * z) - 3.0f));
        Y[13] = SH_C3C * (x * z5);
        Y[14] = SH_C3E * (z * (x * x - y * y));
        Y[15] = SH_C3A * (x * (x * x - 3.0f * (y * y)));
    }
}

// sum_b w[b] grad Y_b at (x, y, z): the Cartesian gradient of the
// polynomials above (their tangential part is what the normalisation of
// the direction passes on)
template <int L>
__device__ __forceinline__ void sh_grad(float x, float y, float z,
                                        const float (&w)[(L + 1) * (L + 1)], float (&g)[3]) {
    g[0] = 0.0f;
    g[1] = 0.0f;
    g[2] = 0.0f;
    if constexpr (L >= 1) {
        g[0] += SH_C1 * w[3];
        g[1] += SH_C1 * w[1];
        g[2] += SH_C1 * w[2];
    }
    if constexpr (L >= 2) {
        g[0] += SH_C2A * (w[4] * y + w[7] * z) + 2.0f * SH_C2C * w[8] * x;
        g[1] += SH_C2A * (w[4] * x + w[5] * z) - 2.0f * SH_C2C * w[8] * y;
        g[2] += SH_C2A * (w[5] * y + w[7] * x) + 6.0f * SH_C2B * w[6] * z;
    }
    if constexpr (L >= 3) {
        const float z5 = 5.0f * (z * z) - 1.0f;
        const float xx_yy = 3.0f * (x * x) - 3.0f * (y * y);
        g[0] += SH_C3A * (6.0f * w[9] * (x * y) + w[15] * xx_yy) + SH_C3B * w[10] * (y * z) +
                SH_C3C * w[13] * z5 + 2.0f * SH_C3E * w[14] * (x * z);
        g[1] += SH_C3A * (w[9] * xx_yy - 6.0f * w[15] * (x * y)) + SH_C3B * w[10] * (x * z) +
                SH_C3C * w[11] * z5 - 2.0f * SH_C3E * w[14] * (y * z);
        g[2] += SH_C3B * w[10] * (x * y) + 10.0f * SH_C3C * z * (w[11] * y + w[13] * x) +
                SH_C3D * w[12] * (15.0f * (z * z) - 3.0f) + SH_C3E * w[14] * (x * x - y * y);
    }
}

// Unnormalised viewing direction v = mu_c - C (C = -R^T t the camera
// centre), its length and unit direction.
__device__ __forceinline__ void view_dir(const gs4d_view &V, const float (&mu)[3], float (&d)[3],
                                         float &len) {
    const float *Rt = V.Rt;
    float v[3];
    for (int j = 0; j < 3; ++j) {
        const float Cj = -(Rt[j] * Rt[3] + Rt[4 + j] * Rt[7] + Rt[8 + j] * Rt[11]);
        v[j] = mu[j] - Cj;
    }
    len = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const float il = 1.0f / len;
    for (int j = 0; j < 3; ++j) d[j] = v[j] * il;
}

__device__ __forceinline__ float sch_time_factor(int f, float t, float period) {
    return f == 0 ? 1.0f : cosf((6.28318530717958648f * (float)f) * t / period);
}

template <int L>
__global__ void __launch_bounds__(256)
preprocess_sch_fwd_kernel(const float *__restrict__ P, const float *__restrict__ coef, int64_t n,
                          int n_freq, float period, ViewPack vp, float4 *__restrict__ rec,
                          int4 *__restrict__ rect, int32_t *__restrict__ touched) {
    constexpr int NB = (L + 1) * (L + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int vi = blockIdx.y;
    if (g >= n) return;
    float p[20];
#pragma unroll
    for (int k = 0; k < 17; ++k) p[k] = P[(int64_t)k * n + g];
    p[17] = p[18] = p[19] = 0.0f;   // the colour comes from the coefficients
    Slice S;
    int4 rc = make_int4(0, 0, 0, 0);
    const gs4d_view &V = vp.v[vi];
    const int vis = slice_project(p, V, S, &rc);
    const int64_t o = (int64_t)vi * n + g;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    int tt = 0;
    if (vis) {
        float d[3], len;
        view_dir(V, S.mu, d, len);
        float Y[NB];
        sh_eval<L>(d[0], d[1], d[2], Y);
        float col[3] = {0.0f, 0.0f, 0.0f};
        for (int f = 0; f <= n_freq; ++f) {
            const float tf = sch_time_factor(f, V.t, period);
            const float *cf = coef + (int64_t)(f * NB) * 3 * n + g;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float w = tf * Y[b];
#pragma unroll
                for (int c = 0; c < 3; ++c) col[c] += w * cf[(int64_t)(3 * b + c) * n];
            }
        }
        if (isfinite(col[0]) && isfinite(col[1]) && isfinite(col[2])) {
            r0 = make_float4(S.mx, S.my, S.ca, S.cb);
            r1 = make_float4(S.cc, S.ot, S.xc[2], S.hx);
            r2 = make_float4(col[0], col[1], col[2], S.hy);
            tt = (rc.z - rc.x) * (rc.w - rc.y);
        } else {
            rc = make_int4(0, 0, 0, 0);   // non-finite coefficients: culled
        }
    } else {
        rc = make_int4(0, 0, 0, 0);
    }
    rec[3 * o + 0] = r0;
    rec[3 * o + 1] = r1;
    rec[3 * o + 2] = r2;
    rect[o] = rc;
    touched[o] = tt;
}

// Backward of the SCH form, summed over views: the colour gradient g_c of
// each (view, Gaussian) gives d coef_{b,c} = Z_b g_c and, through the
// viewing direction, d mu_c = (I - d d^T) / |v| sum_b w_b grad Y_b with
// w_b = sum_n cos(.) sum_c g_c coef; that joins the projection's d mu_c
// ahead of the rotor form's chain rule.  dparams rows 17-19 are zero.
template <int L>
__global__ void __launch_bounds__(128, 3)
preprocess_sch_bwd_kernel(const float *__restrict__ P, const float *__restrict__ coef, int64_t n,
                          int n_freq, float period, ViewPack vp,
                          const int32_t *__restrict__ touched, const float *__restrict__ grad2d,
                          float *__restrict__ dP, float *__restrict__ dcoef) {
    constexpr int NB = (L + 1) * (L + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float p[20];
#pragma unroll
    for (int k = 0; k < 17; ++k) p[k] = P[(int64_t)k * n + g];
    p[17] = p[18] = p[19] = 0.0f;
    float acc[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) acc[k] = 0.0f;
    const int64_t rows = (int64_t)(n_freq + 1) * NB * 3;
    bool first = true;

    for (int vi = 0; vi < vp.n_views; ++vi) {
        const int64_t o = (int64_t)vi * n + g;
        if (touched[o] == 0) continue;
        const gs4d_view &V = vp.v[vi];
        Slice S;
        if (!slice_project(p, V, S, nullptr)) continue;
        float G[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = grad2d[o * 9 + k];
        float Gmu[3], GSc[3][3];
        project_bwd(V, S, G, Gmu, GSc);

        float d[3], len;
        view_dir(V, S.mu, d, len);
        float Y[NB], w[NB];
        sh_eval<L>(d[0], d[1], d[2], Y);
#pragma unroll
        for (int b = 0; b < NB; ++b) w[b] = 0.0f;
        for (int f = 0; f <= n_freq; ++f) {
            const float tf = sch_time_factor(f, V.t, period);
            const int64_t base = (int64_t)(f * NB) * 3 * n + g;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float wc = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t idx = base + (int64_t)(3 * b + c) * n;
                    wc += G[6 + c] * coef[idx];
                    const float dv = (tf * Y[b]) * G[6 + c];
                    dcoef[idx] = first ? dv : dcoef[idx] + dv;
                }
                w[b] += tf * wc;
            }
        }
        first = false;
        float gd[3];
        sh_grad<L>(d[0], d[1], d[2], w, gd);
        const float radial = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
        const float il = 1.0f / len;
        for (int j = 0; j < 3; ++j) Gmu[j] += (gd[j] - d[j] * radial) * il;

        rotor_chain(S, Gmu, GSc, G[5], acc);
    }
    if (first)
        for (int64_t r = 0; r < rows; ++r) dcoef[r * n + g] = 0.0f;
#pragma unroll
    for (int k = 0; k < 20; ++k) dP[(int64_t)k * n + g] = acc[k];
}

// Coefficients whose colour is the constant rgb: only the n = 0, l = 0
// basis, coef = rgb / Y_00 = 2 sqrt(pi) rgb; every other row zero.
__global__ void __launch_bounds__(256)
sch_from_rgb_kernel(const float *__restrict__ rgb, int64_t rgb_stride, int64_t n, int64_t rows,
                    float *__restrict__ coef) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    for (int c = 0; c < 3; ++c) coef[(int64_t)c * n + g] = rgb[c * rgb_stride + g] / SH_C0;
    for (int64_t r = 3; r < rows; ++r) coef[r * n + g] = 0.0f;
}

}  // namespace

}  // namespace gs4d

using namespace gs4d;

extern "C" int gs4d_preprocess(const float *params, int64_t n, const gs4d_view *views,
                               int32_t n_views, float *rec, int32_t *rect, int32_t *touched,
                               void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_REQUIRE(n >= 0, "gs4d_preprocess: n < 0");
    GS4D_REQUIRE(n <= (int64_t)0x7fffffff, "gs4d_preprocess: n >= 2^31");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && rec && rect && touched, "gs4d_preprocess: null pointer");
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
    preprocess_fwd_kernel<<<grid, 256, 0, as_stream(stream)>>>(
        params, n, vp, reinterpret_cast<float4 *>(rec), reinterpret_cast<int4 *>(rect), touched);
    GS4D_LAUNCH_CHECK("gs4d_preprocess");
    return GS4D_OK;
}

extern "C" int gs4d_preprocess_bwd(const float *params, int64_t n, const gs4d_view *views,
                                   int32_t n_views, const int32_t *touched, const float *grad2d,
                                   float *dparams, void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_preprocess_bwd: n out of range");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && touched && grad2d && dparams, "gs4d_preprocess_bwd: null pointer");
    const unsigned blocks = (unsigned)((n + 127) / 128);
    preprocess_bwd_kernel<<<blocks, 128, 0, as_stream(stream)>>>(params, n, vp, touched, grad2d,
                                                                 dparams);
    GS4D_LAUNCH_CHECK("gs4d_preprocess_bwd");
    return GS4D_OK;
}

extern "C" int gs4d_preprocess_iso(const float *params, int64_t n, const gs4d_view *views,
                                   int32_t n_views, float *rec, int32_t *rect, int32_t *touched,
                                   void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_REQUIRE(n >= 0, "gs4d_preprocess_iso: n < 0");
    GS4D_REQUIRE(n <= (int64_t)0x7fffffff, "gs4d_preprocess_iso: n >= 2^31");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && rec && rect && touched, "gs4d_preprocess_iso: null pointer");
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
    preprocess_iso_fwd_kernel<<<grid, 256, 0, as_stream(stream)>>>(
        params, n, vp, reinterpret_cast<float4 *>(rec), reinterpret_cast<int4 *>(rect), touched);
    GS4D_LAUNCH_CHECK("gs4d_preprocess_iso");
    return GS4D_OK;
}

extern "C" int gs4d_preprocess_iso_bwd(const float *params, int64_t n, const gs4d_view *views,
                                       int32_t n_views, const int32_t *touched,
                                       const float *grad2d, float *dparams, void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_preprocess_iso_bwd: n out of range");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && touched && grad2d && dparams, "gs4d_preprocess_iso_bwd: null pointer");
    const unsigned blocks = (unsigned)((n + 127) / 128);
    preprocess_iso_bwd_kernel<<<blocks, 128, 0, as_stream(stream)>>>(params, n, vp, touched,
                                                                     grad2d, dparams);
    GS4D_LAUNCH_CHECK("gs4d_preprocess_iso_bwd");
    return GS4D_OK;
}

namespace {
int check_sch(const gs4d_sch *sch, const char *what) {
    GS4D_REQUIRE(sch != nullptr, "%s: null gs4d_sch", what);
    GS4D_REQUIRE(sch->degree >= 0 && sch->degree <= GS4D_SCH_MAX_DEGREE,
                 "%s: SCH degree %d outside [0, %d]", what, sch->degree, GS4D_SCH_MAX_DEGREE);
    GS4D_REQUIRE(sch->n_freq >= 0 && sch->n_freq <= GS4D_SCH_MAX_FREQ,
                 "%s: SCH temporal frequencies %d outside [0, %d]", what, sch->n_freq,
                 GS4D_SCH_MAX_FREQ);
    GS4D_REQUIRE(sch->period > 0.0f && std::isfinite(sch->period), "%s: SCH period must be > 0", what);
    GS4D_REQUIRE(sch->reserved == 0, "%s: gs4d_sch.reserved must be 0", what);
    return GS4D_OK;
}
}  // namespace

extern "C" int64_t gs4d_sch_rows(int32_t degree, int32_t n_freq) {
    if (degree < 0 || degree > GS4D_SCH_MAX_DEGREE || n_freq < 0 || n_freq > GS4D_SCH_MAX_FREQ)
        return -1;
    return (int64_t)3 * (n_freq + 1) * (degree + 1) * (degree + 1);
}

extern "C" int gs4d_preprocess_sch(const float *params, const float *coef, int64_t n,
                                   const gs4d_sch *sch, const gs4d_view *views, int32_t n_views,
                                   float *rec, int32_t *rect, int32_t *touched, void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_TRY(check_sch(sch, "gs4d_preprocess_sch"));
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_preprocess_sch: n out of range");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && coef && rec && rect && touched, "gs4d_preprocess_sch: null pointer");
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_views);
    hipStream_t st = as_stream(stream);
    float4 *r4 = reinterpret_cast<float4 *>(rec);
    int4 *q4 = reinterpret_cast<int4 *>(rect);
    switch (sch->degree) {
    case 0: preprocess_sch_fwd_kernel<0><<<grid, 256, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, r4, q4, touched); break;
    case 1: preprocess_sch_fwd_kernel<1><<<grid, 256, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, r4, q4, touched); break;
    case 2: preprocess_sch_fwd_kernel<2><<<grid, 256, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, r4, q4, touched); break;
    default: preprocess_sch_fwd_kernel<3><<<grid, 256, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, r4, q4, touched); break;
    }
    GS4D_LAUNCH_CHECK("gs4d_preprocess_sch");
    return GS4D_OK;
}

extern "C" int gs4d_preprocess_sch_bwd(const float *params, const float *coef, int64_t n,
                                       const gs4d_sch *sch, const gs4d_view *views,
                                       int32_t n_views, const int32_t *touched,
                                       const float *grad2d, float *dparams, float *dcoef,
                                       void *stream) {
    ViewPack vp;
    GS4D_TRY(make_view_pack(views, n_views, &vp));
    GS4D_TRY(check_sch(sch, "gs4d_preprocess_sch_bwd"));
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_preprocess_sch_bwd: n out of range");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(params && coef && touched && grad2d && dparams && dcoef,
                 "gs4d_preprocess_sch_bwd: null pointer");
    const unsigned blocks = (unsigned)((n + 127) / 128);
    hipStream_t st = as_stream(stream);
    switch (sch->degree) {
    case 0: preprocess_sch_bwd_kernel<0><<<blocks, 128, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, touched, grad2d, dparams, dcoef); break;
    case 1: preprocess_sch_bwd_kernel<1><<<blocks, 128, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, touched, grad2d, dparams, dcoef); break;
    case 2: preprocess_sch_bwd_kernel<2><<<blocks, 128, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, touched, grad2d, dparams, dcoef); break;
    default: preprocess_sch_bwd_kernel<3><<<blocks, 128, 0, st>>>(params, coef, n, sch->n_freq, sch->period, vp, touched, grad2d, dparams, dcoef); break;
    }
    GS4D_LAUNCH_CHECK("gs4d_preprocess_sch_bwd");
    return GS4D_OK;
}

extern "C" int gs4d_sch_from_rgb(const float *rgb, int64_t rgb_stride, int64_t n,
                                 const gs4d_sch *sch, float *coef, void *stream) {
    GS4D_TRY(check_sch(sch, "gs4d_sch_from_rgb"));
    GS4D_REQUIRE(n >= 0 && n <= (int64_t)0x7fffffff, "gs4d_sch_from_rgb: n out of range");
    GS4D_REQUIRE(rgb_stride >= n, "gs4d_sch_from_rgb: rgb_stride < n");
    if (n == 0) return GS4D_OK;
    GS4D_REQUIRE(rgb && coef, "gs4d_sch_from_rgb: null pointer");
    const int64_t rows = gs4d_sch_rows(sch->degree, sch->n_freq);
    sch_from_rgb_kernel<<<(unsigned)((n + 255) / 256), 256, 0, as_stream(stream)>>>(
        rgb, rgb_stride, n, rows, coef);
    GS4D_LAUNCH_CHECK("gs4d_sch_from_rgb");
    return GS4D_OK;
}
