// Backward preprocess, optimiser step, relocation and mature.
//
// k_preprocess_bwd: per optimisable slot of the window set A, the chain rule
// from the per-view record gradients d(u, v, A, B, C, o, rgb) to the slot's
// parameters, summed over every view of the plan in which the slot is live
// (Algorithm 1's backward; frozen slots get none, Sec. 4.2).  FP64, so the
// clamp decisions (FoV clamp of the Jacobian, rgb >= 0) are those of the
// forward.  No atomics: one thread owns one slot.
//
// k_adam_sgld: Adam over A with the adaptive mean-gradient scaling of
// Sec. 4.5.1, then SGLD noise on the means (Algorithm 1's noise line,
// Sec. 4.4), Philox4x32-10 normals.
//
// Relocation (Sec. 3.2): dead = logit below fl32(logit(0.005)); sources
// drawn from the alive slots with integer opacity weights through an exact
// 64-bit CDF search; the copies and the sources are rescaled.
//
// Mature (Algorithm 1's mature): snapshot, pack, re-arm.
#include "swgs_internal.h"

namespace swgs {
namespace {

constexpr int kBlock = 256;

// ------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): 10 rounds; multipliers 0xD2511F53 and
// 0xCD9E8D57, key increments 0x9E3779B9 and 0xBB67AE85.
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t h0 = __umulhi(0xD2511F53u, c.x), l0 = 0xD2511F53u * c.x;
        const uint32_t h1 = __umulhi(0xCD9E8D57u, c.z), l1 = 0xCD9E8D57u * c.z;
        c = make_uint4(h1 ^ c.y ^ k.x, l1, h0 ^ c.w ^ k.y, l0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// Real SH basis (degree <= 3, 3DGS sign/order) in FP32 at a unit direction.
__device__ __forceinline__ void sh_basis32(int deg, float x, float y, float z, float *Y) {
    Y[0] = 0.28209479177387814f;
    if (deg < 1) return;
    const float c1 = 0.4886025119029199f;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = -1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
    Y[10] = 2.890611442640554f * x * y * z;
    Y[11] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.445305721320277f * z * (xx - yy);
    Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// Gradient w.r.t. (x, y, z) (components independent) of sum_k w[k] Y_k.
__device__ __forceinline__ void sh_weighted_grad(int deg, float x, float y, float z, const float *w, float &gx,
                                                 float &gy, float &gz) {
    gx = gy = gz = 0.0f;
    if (deg < 1) return;
    const float c1 = 0.4886025119029199f;
    gy -= c1 * w[1];
    gz += c1 * w[2];
    gx -= c1 * w[3];
    if (deg < 2) return;
    const float a = 1.0925484305920792f, b = 0.31539156525252005f, c = 0.5462742152960396f;
    gx += a * y * w[4];                gy += a * x * w[4];
    gy -= a * z * w[5];                gz -= a * y * w[5];
    gx -= 2.0f * b * x * w[6];         gy -= 2.0f * b * y * w[6];        gz += 4.0f * b * z * w[6];
    gx -= a * z * w[7];                gz -= a * x * w[7];
    gx += 2.0f * c * x * w[8];         gy -= 2.0f * c * y * w[8];
    if (deg < 3) return;
    const float e = 0.5900435899266435f, f = 2.890611442640554f, h = 0.4570457994644658f;
    const float m = 0.3731763325901154f, n = 1.445305721320277f;
    const float xx = x * x, yy = y * y, zz = z * z;
    gx -= 6.0f * e * x * y * w[9];     gy -= 3.0f * e * (xx - yy) * w[9];
    gx += f * y * z * w[10];           gy += f * x * z * w[10];          gz += f * x * y * w[10];
    gx += 2.0f * h * x * y * w[11];    gy -= h * (4.0f * zz - xx - 3.0f * yy) * w[11];  gz -= 8.0f * h * y * z * w[11];
    gx -= 6.0f * m * x * z * w[12];    gy -= 6.0f * m * y * z * w[12];   gz += m * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
    gx -= h * (4.0f * zz - 3.0f * xx - yy) * w[13];  gy += 2.0f * h * x * y * w[13];  gz -= 8.0f * h * x * z * w[13];
    gx += 2.0f * n * x * z * w[14];    gy -= 2.0f * n * y * z * w[14];   gz += n * (xx - yy) * w[14];
    gx -= 3.0f * e * (xx - yy) * w[15]; gy += 6.0f * e * x * y * w[15];
}

// Colour part of the backward preprocess (FP32): SH coefficient gradients
// and the view-direction contribution to the mean gradient, summed over the
// views where the slot is live; runs after k_prebwd_geom and adds to its
// mean gradient.  Three lanes per slot, lane c taking colour channel c (21
// slots per wave, lane 63 idle): the channel's SH coefficient gradients and
// its part of the view-direction term, which is linear in the channel's
// weights; the three parts are added in channel order across the lanes.
constexpr int kColorSlotsPerWave = 21;

template <int DEG>
__global__ void __launch_bounds__(kBlock)
k_prebwd_color(const float *__restrict__ params, int n_slots, int num_gs, const uint32_t *__restrict__ listA,
               uint32_t nA, const GroupDev *__restrict__ groups, int n_groups,
               const int32_t *__restrict__ group_views, const ViewDev *__restrict__ views,
               const int32_t *__restrict__ pos_of, const uint32_t *__restrict__ tile_count,
               const uint8_t *__restrict__ cflags, const float *__restrict__ rec_grad,
               float *__restrict__ grads) {
    constexpr int nk = (DEG + 1) * (DEG + 1);
    const int lane = threadIdx.x & 63, q = lane / 3, c = lane - 3 * q;
    const uint32_t a = ((blockIdx.x * kBlock + threadIdx.x) >> 6) * kColorSlotsPerWave + (uint32_t)q;
    // lanes without a slot work on the last one and store nothing (every
    // lane reaches the cross-lane sums)
    const bool act = lane < 3 * kColorSlotsPerWave && a < nA;
    const size_t S = (size_t)n_slots, NG = (size_t)num_gs;
    const uint32_t slot = listA[act ? a : nA - 1];
    const float mx = params[slot], my = params[S + slot], mz = params[2 * S + slot];
    float f[nk], dsh[nk];
#pragma unroll
    for (int k = 0; k < nk; ++k) {
        f[k] = params[(11 + 3 * k + c) * S + slot];
        dsh[k] = 0.0f;
    }
    float dm0 = 0.0f, dm1 = 0.0f, dm2 = 0.0f;
    for (int g = 0; g < n_groups; ++g) {
        const int32_t j = pos_of[(size_t)g * NG + slot];
        if (j < 0) continue;
        const GroupDev G = groups[g];
        for (int kv = 0; kv < G.n_views; ++kv) {
            const ViewDev &V = views[group_views[G.view_first + kv]];
            const uint32_t r = V.rec_base + (uint32_t)j;
            if (tile_count[r] == 0) continue;                 // culled in this view
            // rgb_c = max(0, sum_k Y_k f_kc + 1/2); a clamped channel passes nothing
            const float gc = ((cflags[r] >> c) & 1u) ? 0.0f : rec_grad[9 * (size_t)r + 6 + c];
            const float dxv = mx - (float)V.campos[0], dyv = my - (float)V.campos[1], dzv = mz - (float)V.campos[2];
            const float il = rsqrtf(dxv * dxv + dyv * dyv + dzv * dzv);
            const float hx = dxv * il, hy = dyv * il, hz = dzv * il;
            float Y[16], wk[16];
            sh_basis32(DEG, hx, hy, hz, Y);
#pragma unroll
            for (int k = 0; k < nk; ++k) {
                dsh[k] += Y[k] * gc;
                wk[k] = f[k] * gc;
            }
            float gx, gy, gz;
            sh_weighted_grad(DEG, hx, hy, hz, wk, gx, gy, gz);
            // d = dir / |dir|: d dir = (I - d d^T) g / |dir|
            const float dot = gx * hx + gy * hy + gz * hz;
            dm0 += (gx - hx * dot) * il;
            dm1 += (gy - hy * dot) * il;
            dm2 += (gz - hz * dot) * il;
        }
    }
    // the slot's direction term: its channels' parts in channel order
    const int l0 = 3 * q;
    const float t0 = (__shfl(dm0, l0, 64) + __shfl(dm0, l0 + 1, 64)) + __shfl(dm0, l0 + 2, 64);
    const float t1 = (__shfl(dm1, l0, 64) + __shfl(dm1, l0 + 1, 64)) + __shfl(dm1, l0 + 2, 64);
    const float t2 = (__shfl(dm2, l0, 64) + __shfl(dm2, l0 + 1, 64)) + __shfl(dm2, l0 + 2, 64);
    if (!act) return;
    if (c == 0) {
        grads[slot] += t0;
        grads[NG + slot] += t1;
        grads[2 * NG + slot] += t2;
    }
#pragma unroll
    for (int k = 0; k < nk; ++k) grads[(11 + 3 * k + c) * NG + slot] = dsh[k];
}

// Geometry part of the backward preprocess (FP64): projected mean, conic
// and opacity gradients of every live view chained to mean, log-scale,
// quaternion and opacity logit; plus the regulariser and its sums.
__global__ void __launch_bounds__(kBlock)
k_prebwd_geom(const float *__restrict__ params, int n_slots, int num_gs, const uint32_t *__restrict__ listA,
              uint32_t nA, const GroupDev *__restrict__ groups, int n_groups,
              const int32_t *__restrict__ group_views, const ViewDev *__restrict__ views,
              const int32_t *__restrict__ pos_of, const uint32_t *__restrict__ tile_count,
              const uint8_t *__restrict__ cflags, const float *__restrict__ rec_grad,
              float *__restrict__ grads, int add_reg, double reg_o, double reg_s, double *__restrict__ reg_part) {
    const uint32_t a = blockIdx.x * kBlock + threadIdx.x;
    double rsig = 0.0, rscale = 0.0;
    if (a < nA) {
        const size_t S = (size_t)n_slots, NG = (size_t)num_gs;
        const uint32_t slot = listA[a];
        const double mx = params[slot], my = params[S + slot], mz = params[2 * S + slot];
        // Sigma = M M^T, M = R(q) diag(e^s)
        double M[9], Sg[6];   // Sg: 00 01 02 11 12 22
        {
            const double q0 = params[6 * S + slot], q1 = params[7 * S + slot], q2 = params[8 * S + slot],
                         q3 = params[9 * S + slot];
            const double qi = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
            const double w = q0 * qi, x = q1 * qi, y = q2 * qi, z = q3 * qi;
            const double s0 = exp((double)params[3 * S + slot]), s1 = exp((double)params[4 * S + slot]),
                         s2 = exp((double)params[5 * S + slot]);
            M[0] = (1.0 - 2.0 * (y * y + z * z)) * s0; M[1] = 2.0 * (x * y - w * z) * s1; M[2] = 2.0 * (x * z + w * y) * s2;
            M[3] = 2.0 * (x * y + w * z) * s0; M[4] = (1.0 - 2.0 * (x * x + z * z)) * s1; M[5] = 2.0 * (y * z - w * x) * s2;
            M[6] = 2.0 * (x * z - w * y) * s0; M[7] = 2.0 * (y * z + w * x) * s1; M[8] = (1.0 - 2.0 * (x * x + y * y)) * s2;
            Sg[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
            Sg[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
            Sg[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
            Sg[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
            Sg[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
            Sg[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
        }
        const double op = 1.0 / (1.0 + exp(-(double)params[10 * S + slot]));
        double dmu0 = 0, dmu1 = 0, dmu2 = 0, dlogit = 0.0;
        double H[6] = {0, 0, 0, 0, 0, 0};   // symmetric dL/dSigma

        for (int g = 0; g < n_groups; ++g) {
            const int32_t j = pos_of[(size_t)g * NG + slot];
            if (j < 0) continue;
            const GroupDev G = groups[g];
            for (int kv = 0; kv < G.n_views; ++kv) {
                const ViewDev &V = views[group_views[G.view_first + kv]];
                const uint32_t r = V.rec_base + (uint32_t)j;
                if (tile_count[r] == 0) continue;                 // culled in this view
                const uint32_t fl = cflags[r];
                dlogit += (double)rec_grad[9 * (size_t)r + 5] * op * (1.0 - op);
                const double px = V.R[0] * mx + V.R[1] * my + V.R[2] * mz + V.t[0];
                const double py = V.R[3] * mx + V.R[4] * my + V.R[5] * mz + V.t[1];
                const double pz = V.R[6] * mx + V.R[7] * my + V.R[8] * mz + V.t[2];
                const double iz = 1.0 / pz;
                const bool clx = (fl & 8u) != 0, cly = (fl & 16u) != 0;
                const double txr = px * iz, tyr = py * iz;
                const double tx = clx ? (txr < 0 ? -V.limx : V.limx) : txr;
                const double ty = cly ? (tyr < 0 ? -V.limy : V.limy) : tyr;
                const double J00 = V.fx * iz, J02 = -V.fx * tx * iz, J11 = V.fy * iz, J12 = -V.fy * ty * iz;
                double T0[3], T1[3];
                for (int c = 0; c < 3; ++c) {
                    T0[c] = J00 * V.R[c] + J02 * V.R[6 + c];
                    T1[c] = J11 * V.R[3 + c] + J12 * V.R[6 + c];
                }
                const double A0[3] = {Sg[0] * T0[0] + Sg[1] * T0[1] + Sg[2] * T0[2],
                                      Sg[1] * T0[0] + Sg[3] * T0[1] + Sg[4] * T0[2],
                                      Sg[2] * T0[0] + Sg[4] * T0[1] + Sg[5] * T0[2]};
                const double B0[3] = {Sg[0] * T1[0] + Sg[1] * T1[1] + Sg[2] * T1[2],
                                      Sg[1] * T1[0] + Sg[3] * T1[1] + Sg[4] * T1[2],
                                      Sg[2] * T1[0] + Sg[4] * T1[1] + Sg[5] * T1[2]};
                const double ca = T0[0] * A0[0] + T0[1] * A0[1] + T0[2] * A0[2] + 0.3;
                const double cb = T0[0] * B0[0] + T0[1] * B0[1] + T0[2] * B0[2];
                const double cc = T1[0] * B0[0] + T1[1] * B0[1] + T1[2] * B0[2] + 0.3;
                const double det = ca * cc - cb * cb;
                // conic (A, B, C) = (c, -b, a) / det
                const double i2 = 1.0 / (det * det);
                const double gA = rec_grad[9 * (size_t)r + 2], gB = rec_grad[9 * (size_t)r + 3], gC = rec_grad[9 * (size_t)r + 4];
                const double dca = (-cc * cc * gA + cb * cc * gB - cb * cb * gC) * i2;
                const double dcb = (2.0 * cb * cc * gA - (ca * cc + cb * cb) * gB + 2.0 * ca * cb * gC) * i2;
                const double dcc = (-cb * cb * gA + ca * cb * gB - ca * ca * gC) * i2;
                // dL/dSigma summed over views: 2 dca T0 T0^T + dcb (T0 T1^T + T1 T0^T) + 2 dcc T1 T1^T
                H[0] += 2.0 * (dca * T0[0] * T0[0] + dcb * T0[0] * T1[0] + dcc * T1[0] * T1[0]);
                H[1] += 2.0 * dca * T0[0] * T0[1] + dcb * (T0[0] * T1[1] + T1[0] * T0[1]) + 2.0 * dcc * T1[0] * T1[1];
                H[2] += 2.0 * dca * T0[0] * T0[2] + dcb * (T0[0] * T1[2] + T1[0] * T0[2]) + 2.0 * dcc * T1[0] * T1[2];
                H[3] += 2.0 * (dca * T0[1] * T0[1] + dcb * T0[1] * T1[1] + dcc * T1[1] * T1[1]);
                H[4] += 2.0 * dca * T0[1] * T0[2] + dcb * (T0[1] * T1[2] + T1[1] * T0[2]) + 2.0 * dcc * T1[1] * T1[2];
                H[5] += 2.0 * (dca * T0[2] * T0[2] + dcb * T0[2] * T1[2] + dcc * T1[2] * T1[2]);
                double dT0[3], dT1[3];
                for (int c = 0; c < 3; ++c) {
                    dT0[c] = 2.0 * dca * A0[c] + dcb * B0[c];
                    dT1[c] = dcb * A0[c] + 2.0 * dcc * B0[c];
                }
                // T = J R: dJ_rk = sum_c dT_rc R_kc
                const double dJ00 = dT0[0] * V.R[0] + dT0[1] * V.R[1] + dT0[2] * V.R[2];
                const double dJ02 = dT0[0] * V.R[6] + dT0[1] * V.R[7] + dT0[2] * V.R[8];
                const double dJ11 = dT1[0] * V.R[3] + dT1[1] * V.R[4] + dT1[2] * V.R[5];
                const double dJ12 = dT1[0] * V.R[6] + dT1[1] * V.R[7] + dT1[2] * V.R[8];
                double dpx = 0, dpy = 0, dpz = 0;
                dpz += (-dJ00 * V.fx + dJ02 * V.fx * tx - dJ11 * V.fy + dJ12 * V.fy * ty) * iz * iz;
                const double dtx = -dJ02 * V.fx * iz, dty = -dJ12 * V.fy * iz;
                if (!clx) { dpx += dtx * iz; dpz -= dtx * px * iz * iz; }
                if (!cly) { dpy += dty * iz; dpz -= dty * py * iz * iz; }
                // projected mean
                const double gu = rec_grad[9 * (size_t)r], gv = rec_grad[9 * (size_t)r + 1];
                dpx += gu * V.fx * iz;
                dpz -= gu * V.fx * px * iz * iz;
                dpy += gv * V.fy * iz;
                dpz -= gv * V.fy * py * iz * iz;
                dmu0 += V.R[0] * dpx + V.R[3] * dpy + V.R[6] * dpz;
                dmu1 += V.R[1] * dpx + V.R[4] * dpy + V.R[7] * dpz;
                dmu2 += V.R[2] * dpx + V.R[5] * dpy + V.R[8] * dpz;
            }
        }
        // Sigma = M M^T: dM = Hs M with Hs the symmetric matrix of H; M = R(q) diag(sc)
        const double q0 = params[6 * S + slot], q1 = params[7 * S + slot], q2 = params[8 * S + slot],
                     q3 = params[9 * S + slot];
        const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
        const double sc[3] = {exp((double)params[3 * S + slot]), exp((double)params[4 * S + slot]),
                              exp((double)params[5 * S + slot])};
        const double Hs[9] = {H[0], H[1], H[2], H[1], H[3], H[4], H[2], H[4], H[5]};
        double dRq[9], ds[3];
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int r2 = 0; r2 < 3; ++r2) {
                const double dm = Hs[3 * r2] * M[c] + Hs[3 * r2 + 1] * M[3 + c] + Hs[3 * r2 + 2] * M[6 + c];
                dRq[3 * r2 + c] = dm * sc[c];
                acc += dm * M[3 * r2 + c] / sc[c];     // Rq = M / sc
            }
            ds[c] = acc * sc[c];
        }
        double dq[4];
        dq[0] = 2.0 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
        dq[1] = 2.0 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2.0 * x * dRq[4] - w * dRq[5] + z * dRq[6] +
                       w * dRq[7] - 2.0 * x * dRq[8]);
        dq[2] = 2.0 * (-2.0 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] +
                       z * dRq[7] - 2.0 * y * dRq[8]);
        dq[3] = 2.0 * (-2.0 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2.0 * z * dRq[4] + y * dRq[5] +
                       x * dRq[6] + y * dRq[7]);
        const double qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
        const double qh[4] = {w, x, y, z};
        if (add_reg) {
            dlogit += reg_o * op * (1.0 - op);
            for (int c = 0; c < 3; ++c) ds[c] += reg_s * sc[c];
        }
        rsig = op;
        rscale = sc[0] + sc[1] + sc[2];
        grads[slot] = (float)dmu0;
        grads[NG + slot] = (float)dmu1;
        grads[2 * NG + slot] = (float)dmu2;
        for (int c = 0; c < 3; ++c) grads[(3 + c) * NG + slot] = (float)ds[c];
        for (int k = 0; k < 4; ++k) grads[(6 + k) * NG + slot] = (float)((dq[k] - qh[k] * qd) / qn);
        grads[10 * NG + slot] = (float)dlogit;
    }
    // regulariser sums (for the reported loss)
    __shared__ double red[2][kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) {
        rsig += __shfl_xor(rsig, o, 64);
        rscale += __shfl_xor(rscale, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = rsig;
        red[1][threadIdx.x >> 6] = rscale;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
        for (int w2 = 0; w2 < kBlock / 64; ++w2) { s0 += red[0][w2]; s1 += red[1][w2]; }
        reg_part[2 * blockIdx.x] = s0;
        reg_part[2 * blockIdx.x + 1] = s1;
    }
}

__global__ void __launch_bounds__(256)
k_reg_reduce(const double *__restrict__ part, int nparts, double lo, double ls, double invA,
             const uint32_t *__restrict__ pair_count, double *__restrict__ stats) {
    __shared__ double sa[256], sb[256];
    double a = 0, b = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) { a += part[2 * i]; b += part[2 * i + 1]; }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) { sa[threadIdx.x] += sa[threadIdx.x + s]; sb[threadIdx.x] += sb[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[2] = lo * sa[0] * invA + ls * sb[0] * invA;
        stats[3] = stats[0] + stats[2];
        stats[4] = (double)pair_count[0];
        stats[6] = (double)pair_count[1];
    }
}

// --------------------------------------------------------------- Adam + SGLD
__global__ void __launch_bounds__(kBlock)
k_adam_sgld(float *__restrict__ params, int n_slots, const float *__restrict__ grads, float *__restrict__ m,
            float *__restrict__ v, int num_gs, int F, const uint32_t *__restrict__ listA, uint32_t nA,
            const int32_t *__restrict__ start, swgs_step_cfg cfg, int swin, const StepDev *__restrict__ sd,
            const float *__restrict__ eta) {
    const uint32_t a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nA) return;
    const size_t S = (size_t)n_slots, NG = (size_t)num_gs;
    const uint32_t slot = listA[a];
    const StepDev st = *sd;
    const double t = (double)st.adam_t;
    const float bc1 = (float)(1.0 - pow((double)cfg.beta1, t));
    const float bc2 = (float)(1.0 - pow((double)cfg.beta2, t));
    float gscale = 1.0f;
    if (cfg.grad_scale_base > 0.0f) {
        int wtr = cfg.window_start - start[slot] + swin - 1;
        wtr = wtr < 0 ? 0 : (wtr > swin - 1 ? swin - 1 : wtr);
        gscale = (float)pow((double)cfg.grad_scale_base, (double)wtr / (double)swin);
    }
    for (int r = 0; r < F; ++r) {
        const float lr = r < 3 ? cfg.lr_mean
                       : r < 6 ? cfg.lr_scale
                       : r < 10 ? cfg.lr_quat
                       : r == 10 ? cfg.lr_logit
                       : r < 14 ? cfg.lr_sh_dc : cfg.lr_sh_rest;
        float g = grads[r * NG + slot];
        if (r < 3) g *= gscale;
        const float mm = cfg.beta1 * m[r * NG + slot] + (1.0f - cfg.beta1) * g;
        const float vv = cfg.beta2 * v[r * NG + slot] + (1.0f - cfg.beta2) * g * g;
        m[r * NG + slot] = mm;
        v[r * NG + slot] = vv;
        const float mh = mm / bc1, vh = vv / bc2;
        params[r * S + slot] -= lr * mh / (sqrtf(vh) + cfg.eps);
    }
    if (cfg.noise_lr == 0.0f) return;
    // SGLD noise with the updated covariance and opacity
    float e0, e1, e2;
    if (eta) {
        e0 = eta[slot];
        e1 = eta[NG + slot];
        e2 = eta[2 * NG + slot];
    } else {
        const uint4 x = philox(make_uint4(slot, (uint32_t)st.step, (uint32_t)(st.step >> 32), 0x4E4F4953u),
                               make_uint2((uint32_t)st.seed, (uint32_t)(st.seed >> 32)));
        const float u1 = (float)((x.x >> 8) + 1u) * 5.9604644775390625e-8f;
        const float u2 = (float)(x.y >> 8) * 5.9604644775390625e-8f;
        const float u3 = (float)((x.z >> 8) + 1u) * 5.9604644775390625e-8f;
        const float u4 = (float)(x.w >> 8) * 5.9604644775390625e-8f;
        const float r1 = sqrtf(-2.0f * logf(u1)), r2 = sqrtf(-2.0f * logf(u3));
        const float twopi = 6.283185307179586f;
        e0 = r1 * cosf(twopi * u2);
        e1 = r1 * sinf(twopi * u2);
        e2 = r2 * cosf(twopi * u4);
    }
    float qw = params[6 * S + slot], qx = params[7 * S + slot], qy = params[8 * S + slot], qz = params[9 * S + slot];
    const float qi = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qi; qx *= qi; qy *= qi; qz *= qi;
    const float s0 = expf(params[3 * S + slot]), s1 = expf(params[4 * S + slot]), s2 = expf(params[5 * S + slot]);
    const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                        2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    // Sigma eta = R S^2 R^T eta
    const float w0 = s0 * s0 * (R[0] * e0 + R[3] * e1 + R[6] * e2);
    const float w1 = s1 * s1 * (R[1] * e0 + R[4] * e1 + R[7] * e2);
    const float w2 = s2 * s2 * (R[2] * e0 + R[5] * e1 + R[8] * e2);
    const float o = 1.0f / (1.0f + expf(-params[10 * S + slot]));
    const float gate = 1.0f / (1.0f + expf(cfg.noise_k * (o - cfg.noise_t0)));
    const float coef = cfg.noise_lr * cfg.lr_mean * gate;
    params[0 * S + slot] += coef * (R[0] * w0 + R[1] * w1 + R[2] * w2);
    params[1 * S + slot] += coef * (R[3] * w0 + R[4] * w1 + R[5] * w2);
    params[2 * S + slot] += coef * (R[6] * w0 + R[7] * w1 + R[8] * w2);
}

__global__ void k_set_step(StepDev *sd, int64_t adam_t, uint64_t step, uint64_t seed) {
    sd->adam_t = adam_t;
    sd->step = step;
    sd->seed = seed;
}

// ------------------------------------------------------------------ relocation
__device__ __forceinline__ double softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

// S_N(a) = sum_{i=1..N} sum_{k<i} C(i-1,k) (-1)^k a^{k+1}/sqrt(k+1); summing
// over i first (sum_{i=k+1..N} C(i-1,k) = C(N,k+1)) gives the single sum
// sum_{m=1..N} (-1)^{m-1} C(N,m) a^m / sqrt(m).
__device__ double reloc_SN(int N, double a) {
    double s = 0.0, binom = 1.0, ap = 1.0;
    for (int mm = 1; mm <= N; ++mm) {
        binom = binom * (double)(N - mm + 1) / (double)mm;
        ap *= a;
        const double term = binom * ap / sqrt((double)mm);
        s += (mm & 1) ? term : -term;
    }
    return s;
}

__global__ void __launch_bounds__(kBlock)
k_reloc_flags(const float *__restrict__ params, int n_slots, const uint32_t *__restrict__ listA, uint32_t nA,
              const StepDev *__restrict__ sd, int period, uint32_t *__restrict__ dead, uint64_t *__restrict__ w) {
    const uint32_t a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nA) return;
    const bool on = period > 0 && (sd->step % (uint64_t)period) == 0;
    const float lg = params[10 * (size_t)n_slots + listA[a]];
    const float Ls = -5.293304824724492f;   // fl32(ln(0.005/0.995))
    const bool d = on && lg < Ls;
    dead[a] = d ? 1u : 0u;
    w[a] = (!on || d) ? 0ull : (uint64_t)floor(16777216.0 / (1.0 + exp(-(double)lg)));
}

// inclusive u64 scan, single pass per 2048-chunk + carry chain over chunks
constexpr int kU64Chunk = 2048;
__global__ void __launch_bounds__(kBlock)
k_u64_reduce(const uint64_t *__restrict__ in, uint32_t n, uint64_t *__restrict__ sums) {
    __shared__ uint64_t ws[kBlock / 64];
    uint64_t s = 0;
    const uint32_t lo = blockIdx.x * kU64Chunk;
    for (uint32_t i = lo + threadIdx.x; i < min(n, lo + kU64Chunk); i += kBlock) s += in[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}
__global__ void k_u64_carry(uint64_t *sums, uint32_t nb, uint64_t *total) {
    if (threadIdx.x != 0) return;
    uint64_t c = 0;
    for (uint32_t i = 0; i < nb; ++i) { uint64_t v = sums[i]; sums[i] = c; c += v; }
    *total = c;
}
__global__ void __launch_bounds__(kBlock)
k_u64_write(uint64_t *__restrict__ io, uint32_t n, const uint64_t *__restrict__ sums) {
    __shared__ uint64_t ws[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t carry = sums[blockIdx.x];
    const uint32_t lo = blockIdx.x * kU64Chunk;
    for (uint32_t t0 = lo; t0 < min(n, lo + kU64Chunk); t0 += kBlock) {
        const uint32_t i = t0 + threadIdx.x;
        uint64_t x = i < n ? io[i] : 0;
        for (int o = 1; o < 64; o <<= 1) {
            uint64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) ws[wave] = x;
        __syncthreads();
        uint64_t before = carry;
        for (int w = 0; w < wave; ++w) before += ws[w];
        if (i < n) io[i] = before + x;          // inclusive
        const uint64_t tot = ws[0] + ws[1] + ws[2] + ws[3];
        __syncthreads();
        carry += tot;
    }
}

__global__ void __launch_bounds__(kBlock)
k_reloc_dst(const uint32_t *__restrict__ dead, const uint32_t *__restrict__ dpos, const uint32_t *__restrict__ listA,
            uint32_t nA, int32_t *__restrict__ dst) {
    const uint32_t a = blockIdx.x * kBlock + threadIdx.x;
    if (a < nA && dead[a]) dst[dpos[a]] = (int32_t)listA[a];
}

__global__ void __launch_bounds__(kBlock)
k_reloc_draw(const uint64_t *__restrict__ pref, uint32_t nA, const uint64_t *__restrict__ Wtot,
             const uint32_t *__restrict__ nD, const StepDev *__restrict__ sd, const uint32_t *__restrict__ listA,
             int32_t *__restrict__ src, uint32_t *__restrict__ src_a, uint32_t *__restrict__ cnt) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    const uint64_t W = *Wtot;
    if (j >= *nD || W == 0) return;
    const StepDev st = *sd;
    const uint4 x = philox(make_uint4(j, (uint32_t)st.step, (uint32_t)(st.step >> 32), 0x52454C4Fu),
                           make_uint2((uint32_t)st.seed, (uint32_t)(st.seed >> 32)));
    const uint64_t r = (uint64_t)x.x | ((uint64_t)x.y << 32);
    const uint64_t u = __umul64hi(r, W);
    // first a with pref[a] > u
    uint32_t lo = 0, hi = nA;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pref[mid] > u) hi = mid; else lo = mid + 1;
    }
    src_a[j] = lo;
    src[j] = (int32_t)listA[lo];
    atomicAdd(cnt + lo, 1u);
}

__device__ __forceinline__ void reloc_new(double lg, int N, double &newlogit, double &dscale) {
    const double l1m = -softplus(lg) / (double)N;      // ln(1 - o')
    const double on = -expm1(l1m);                     // o'
    newlogit = log(on) - l1m;
    dscale = -softplus(-lg) - log(reloc_SN(N, on));
}

__global__ void __launch_bounds__(kBlock)
k_reloc_copies(float *__restrict__ params, int n_slots, float *__restrict__ m, float *__restrict__ v, int num_gs,
               int F, const int32_t *__restrict__ dst, const int32_t *__restrict__ src,
               const uint32_t *__restrict__ src_a, const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ nD,
               const uint64_t *__restrict__ Wtot, int n_max) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= *nD || *Wtot == 0) return;
    const size_t S = (size_t)n_slots, NG = (size_t)num_gs;
    const int d = dst[j], s = src[j];
    int N = 1 + (int)cnt[src_a[j]];
    if (N > n_max) N = n_max;
    double nl, dsc;
    reloc_new((double)params[10 * S + s], N, nl, dsc);
    for (int r = 0; r < F; ++r) params[r * S + d] = params[r * S + s];
    params[10 * S + d] = (float)nl;
    for (int c = 0; c < 3; ++c) params[(3 + c) * S + d] = (float)((double)params[(3 + c) * S + s] + dsc);
    for (int r = 0; r < F; ++r) { m[r * NG + d] = 0.0f; v[r * NG + d] = 0.0f; }
}

__global__ void __launch_bounds__(kBlock)
k_reloc_sources(float *__restrict__ params, int n_slots, float *__restrict__ m, float *__restrict__ v, int num_gs,
                int F, const uint32_t *__restrict__ listA, uint32_t nA, const uint32_t *__restrict__ cnt, int n_max) {
    const uint32_t a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nA || cnt[a] == 0) return;
    const size_t S = (size_t)n_slots, NG = (size_t)num_gs;
    const uint32_t s = listA[a];
    int N = 1 + (int)cnt[a];
    if (N > n_max) N = n_max;
    double nl, dsc;
    reloc_new((double)params[10 * S + s], N, nl, dsc);
    params[10 * S + s] = (float)nl;
    for (int c = 0; c < 3; ++c) params[(3 + c) * S + s] = (float)((double)params[(3 + c) * S + s] + dsc);
    for (int r = 0; r < F; ++r) { m[r * NG + s] = 0.0f; v[r * NG + s] = 0.0f; }
}

__global__ void k_reloc_finish(const uint32_t *nD, const uint64_t *Wtot, int32_t *count_out, double *stats) {
    const int32_t c = (*Wtot == 0) ? 0 : (int32_t)*nD;
    if (count_out) *count_out = c;
    if (stats) stats[5] = (double)c;
}

__global__ void k_stats_out(const double *in, const uint32_t *pc, const uint32_t *nA, double *out) {
    for (int i = 0; i < 8; ++i) out[i] = in[i];
    out[4] = (double)pc[0];
    // bit 0: pair capacity overflow; bit 1: live counts differ from the
    // plan's (lifespans changed after plan creation; the lists are stale)
    out[6] = (double)(pc[1] | (pc[3] ? 2u : 0u));
    if (nA) out[7] = (double)nA[0];
}

// -------------------------------------------------------------------- mature
__global__ void __launch_bounds__(kBlock)
k_mature_flags(const int32_t *__restrict__ start, int num_gs, int st, uint32_t *__restrict__ flag) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < num_gs) flag[i] = start[i] < st ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock)
k_mature_pack(float *__restrict__ params, int n_slots, int num_gs, int F, int swin, int sh_degree, int st,
              int32_t *__restrict__ birth, int32_t *__restrict__ start, int32_t *__restrict__ expire,
              const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos, const uint32_t *__restrict__ count,
              uint8_t *__restrict__ record) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t n = *count;
    if (i == 0) {
        int32_t *h = reinterpret_cast<int32_t *>(record);
        h[0] = 0x53475753; h[1] = 1; h[2] = st; h[3] = (int32_t)n;
        h[4] = sh_degree; h[5] = F; h[6] = swin; h[7] = 0;
    }
    if (i >= num_gs || !flag[i]) return;
    const size_t S = (size_t)n_slots;
    const uint32_t k = pos[i];
    uint32_t *slots = reinterpret_cast<uint32_t *>(record + 32);
    int32_t *lb = reinterpret_cast<int32_t *>(record + 32 + 4 * (size_t)n);
    float *pr = reinterpret_cast<float *>(record + 32 + 16 * (size_t)n);
    slots[k] = (uint32_t)i;
    const int32_t b = birth[i], s = start[i], e = expire[i];
    lb[k] = b;
    lb[n + k] = s;
    lb[2 * (size_t)n + k] = e;
    for (int r = 0; r < F; ++r) {
        const float x = params[r * S + i];
        pr[(size_t)r * n + k] = x;
        params[r * S + num_gs + i] = x;
    }
    birth[num_gs + i] = b;
    start[num_gs + i] = s;
    expire[num_gs + i] = e;
    birth[i] = e;
    start[i] = e;
    expire[i] = e + swin;
}

// Algorithm 2's update: entry k of a mature record goes to slot
// record.slot[k] (slot_base < 0: the slice the record was emitted from) or
// to slot_base + k; parameters and lifespan are overwritten.  Entries whose
// slot is outside the pool are skipped and counted in *bad.
__global__ void __launch_bounds__(kBlock)
k_apply_update(float *__restrict__ params, int n_slots, int F, int32_t *__restrict__ birth,
               int32_t *__restrict__ start, int32_t *__restrict__ expire, const uint8_t *__restrict__ record,
               uint32_t n, int64_t slot_base, uint32_t *__restrict__ bad) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const uint32_t *slots = reinterpret_cast<const uint32_t *>(record + 32);
    const int32_t *lb = reinterpret_cast<const int32_t *>(record + 32 + 4 * (size_t)n);
    const float *pr = reinterpret_cast<const float *>(record + 32 + 16 * (size_t)n);
    const int64_t slot = slot_base < 0 ? (int64_t)slots[k] : slot_base + (int64_t)k;
    if (slot < 0 || slot >= n_slots) {
        atomicAdd(bad, 1u);
        return;
    }
    const size_t S = (size_t)n_slots;
    for (int r = 0; r < F; ++r) params[r * S + (size_t)slot] = pr[(size_t)r * n + k];
    if (birth) birth[slot] = lb[k];
    start[slot] = lb[n + k];
    expire[slot] = lb[2 * (size_t)n + k];
}

}  // namespace

void launch_apply_update(hipStream_t s, const swgs_pool &pool, int F, const uint8_t *record, uint32_t count,
                         int64_t slot_base, uint32_t *bad_slots) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_apply_update, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pool.params,
                       pool.n_slots, F, pool.birth, pool.start, pool.expire, record, count, slot_base, bad_slots);
}

void launch_preprocess_backward(hipStream_t s, const swgs_plan &p, uint8_t *ws, int add_reg,
                                float lambda_o, float lambda_s) {
    const uint32_t nA = p.n_A;
    const int nb = (int)((nA + kBlock - 1) / kBlock);
    if (nb == 0) return;
    const double inv = nA ? 1.0 / (double)nA : 0.0;
#define SWGS_PREBWD_COMMON                                                                                \
    dim3(nb), dim3(kBlock), 0, s, p.pool.params, p.pool.n_slots, p.pool.num_gs,                           \
        wsp<uint32_t>(ws, p, WB_ACTIVE_LIST) + p.list_A_base, nA, wsp<GroupDev>(ws, p, WB_GROUPS),        \
        (int)p.groups.size(), wsp<int32_t>(ws, p, WB_GROUP_VIEWS), wsp<ViewDev>(ws, p, WB_VIEWS),         \
        wsp<int32_t>(ws, p, WB_POS_OF), wsp<uint32_t>(ws, p, WB_TILE_COUNT), wsp<uint8_t>(ws, p, WB_CFLAGS), \
        wsp<float>(ws, p, WB_REC_GRAD), p.pool.grads
    hipLaunchKernelGGL(k_prebwd_geom, SWGS_PREBWD_COMMON, add_reg, (double)lambda_o * inv, (double)lambda_s * inv,
                       wsp<double>(ws, p, WB_REG_PART));
#undef SWGS_PREBWD_COMMON
    // colour: 21 slots per wave, four waves per block
    const uint32_t cw = (nA + kColorSlotsPerWave - 1) / kColorSlotsPerWave;
#define SWGS_PREBWD_COLOR                                                                                 \
    dim3((cw + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, s, p.pool.params, p.pool.n_slots,       \
        p.pool.num_gs, wsp<uint32_t>(ws, p, WB_ACTIVE_LIST) + p.list_A_base, nA,                         \
        wsp<GroupDev>(ws, p, WB_GROUPS), (int)p.groups.size(), wsp<int32_t>(ws, p, WB_GROUP_VIEWS),        \
        wsp<ViewDev>(ws, p, WB_VIEWS), wsp<int32_t>(ws, p, WB_POS_OF), wsp<uint32_t>(ws, p, WB_TILE_COUNT), \
        wsp<uint8_t>(ws, p, WB_CFLAGS), wsp<float>(ws, p, WB_REC_GRAD), p.pool.grads
    switch (p.sh_degree) {
    case 0: hipLaunchKernelGGL(k_prebwd_color<0>, SWGS_PREBWD_COLOR); break;
    case 1: hipLaunchKernelGGL(k_prebwd_color<1>, SWGS_PREBWD_COLOR); break;
    case 2: hipLaunchKernelGGL(k_prebwd_color<2>, SWGS_PREBWD_COLOR); break;
    default: hipLaunchKernelGGL(k_prebwd_color<3>, SWGS_PREBWD_COLOR); break;
    }
#undef SWGS_PREBWD_COLOR
    hipLaunchKernelGGL(k_reg_reduce, dim3(1), dim3(256), 0, s, wsp<double>(ws, p, WB_REG_PART), nb,
                       (double)lambda_o, (double)lambda_s, inv, wsp<uint32_t>(ws, p, WB_PAIR_COUNT),
                       wsp<double>(ws, p, WB_STATS));
}

void launch_adam_sgld(hipStream_t s, const swgs_plan &p, uint8_t *ws, const swgs_step_cfg &cfg,
                      const float *eta) {
    const uint32_t nA = p.n_A;
    if (!nA) return;
    hipLaunchKernelGGL(k_adam_sgld, dim3((nA + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p.pool.params,
                       p.pool.n_slots, p.pool.grads, p.pool.adam_m, p.pool.adam_v, p.pool.num_gs, p.F,
                       wsp<uint32_t>(ws, p, WB_ACTIVE_LIST) + p.list_A_base, nA, p.pool.start, cfg, p.pool.swin,
                       wsp<StepDev>(ws, p, WB_STEP), eta);
}

void launch_relocate(hipStream_t s, const swgs_plan &p, uint8_t *ws, const swgs_step_cfg &cfg,
                     int32_t *dst_out, int32_t *src_out, int32_t *count_out) {
    const uint32_t nA = p.n_A;
    const uint32_t *listA = wsp<uint32_t>(ws, p, WB_ACTIVE_LIST) + p.list_A_base;
    uint64_t *w = wsp<uint64_t>(ws, p, WB_RELOC_W);
    uint32_t *dead = wsp<uint32_t>(ws, p, WB_RELOC_FLAG);
    uint32_t *dpos = dead + nA + 1;
    uint32_t *cnt = wsp<uint32_t>(ws, p, WB_RELOC_CNT);
    uint32_t *src_a = cnt + nA + 1;
    uint32_t *nD = wsp<uint32_t>(ws, p, WB_RELOC_SCAN);
    uint32_t *scan_scratch = nD + 4;
    uint64_t *sums = wsp<uint64_t>(ws, p, WB_RELOC_W) + nA + 1;
    uint64_t *Wtot = sums + (nA + kU64Chunk - 1) / kU64Chunk + 1;
    int32_t *dst = dst_out ? dst_out : wsp<int32_t>(ws, p, WB_RELOC_DST);
    int32_t *src = src_out ? src_out : wsp<int32_t>(ws, p, WB_RELOC_SRC);
    const StepDev *sd = wsp<StepDev>(ws, p, WB_STEP);
    double *stats = wsp<double>(ws, p, WB_STATS);
    if (nA == 0) {
        launch_fill_u32(s, nD, 0, 1);
        hipLaunchKernelGGL(k_u64_carry, dim3(1), dim3(1), 0, s, sums, 0u, Wtot);
        hipLaunchKernelGGL(k_reloc_finish, dim3(1), dim3(1), 0, s, nD, Wtot, count_out, stats);
        return;
    }
    const int nb = (int)((nA + kBlock - 1) / kBlock);
    launch_fill_u32(s, cnt, 0, nA);
    hipLaunchKernelGGL(k_reloc_flags, dim3(nb), dim3(kBlock), 0, s, p.pool.params, p.pool.n_slots, listA, nA, sd,
                       cfg.relocate_period, dead, w);
    exclusive_scan_u32(s, dead, dpos, nA, nD, scan_scratch);
    const uint32_t nbu = (nA + kU64Chunk - 1) / kU64Chunk;
    hipLaunchKernelGGL(k_u64_reduce, dim3(nbu), dim3(kBlock), 0, s, w, nA, sums);
    hipLaunchKernelGGL(k_u64_carry, dim3(1), dim3(1), 0, s, sums, nbu, Wtot);
    hipLaunchKernelGGL(k_u64_write, dim3(nbu), dim3(kBlock), 0, s, w, nA, sums);
    hipLaunchKernelGGL(k_reloc_dst, dim3(nb), dim3(kBlock), 0, s, dead, dpos, listA, nA, dst);
    hipLaunchKernelGGL(k_reloc_draw, dim3(nb), dim3(kBlock), 0, s, w, nA, Wtot, nD, sd, listA, src, src_a, cnt);
    hipLaunchKernelGGL(k_reloc_copies, dim3(nb), dim3(kBlock), 0, s, p.pool.params, p.pool.n_slots, p.pool.adam_m,
                       p.pool.adam_v, p.pool.num_gs, p.F, dst, src, src_a, cnt, nD, Wtot, cfg.reloc_n_max);
    hipLaunchKernelGGL(k_reloc_sources, dim3(nb), dim3(kBlock), 0, s, p.pool.params, p.pool.n_slots, p.pool.adam_m,
                       p.pool.adam_v, p.pool.num_gs, p.F, listA, nA, cnt, cfg.reloc_n_max);
    hipLaunchKernelGGL(k_reloc_finish, dim3(1), dim3(1), 0, s, nD, Wtot, count_out, stats);
}

void launch_set_step(hipStream_t s, uint8_t *ws_step, int64_t adam_t, uint64_t step, uint64_t seed) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, reinterpret_cast<StepDev *>(ws_step), adam_t, step, seed);
}

void launch_stats_out(hipStream_t s, const double *stats, const uint32_t *pair_count, const uint32_t *nA,
                      double *out) {
    hipLaunchKernelGGL(k_stats_out, dim3(1), dim3(1), 0, s, stats, pair_count, nA, out);
}

// mature in two halves: the flags of the slots to mature and their
// exclusive scan (positions, count), then the packing.  Scratch: flag [n+1],
// pos [n+1], then the scan's per-chunk sums.
void launch_mature_count(hipStream_t s, const swgs_pool &pool, int st, uint32_t *flag, uint32_t *pos,
                         uint32_t *d_count) {
    const int n = pool.num_gs;
    uint32_t *scan_scratch = pos + n + 1;
    const int nb = (n + kBlock - 1) / kBlock;
    if (nb == 0) {
        launch_fill_u32(s, d_count, 0, 1);
        return;
    }
    hipLaunchKernelGGL(k_mature_flags, dim3(nb), dim3(kBlock), 0, s, pool.start, n, st, flag);
    exclusive_scan_u32(s, flag, pos, (uint32_t)n, d_count, scan_scratch);
}

void launch_mature_pack(hipStream_t s, const swgs_pool &pool, int F, int st, uint8_t *record, const uint32_t *flag,
                        const uint32_t *pos, const uint32_t *d_count) {
    const int n = pool.num_gs;
    const int nb = (n + kBlock - 1) / kBlock;
    if (nb == 0) return;
    hipLaunchKernelGGL(k_mature_pack, dim3(nb), dim3(kBlock), 0, s, pool.params, pool.n_slots, n, F, pool.swin,
                       pool.sh_degree, st, pool.birth, pool.start, pool.expire, flag, pos, d_count, record);
}

void launch_mature(hipStream_t s, const swgs_pool &pool, int F, int st, uint8_t *record, uint32_t *scratch,
                   uint32_t *d_count) {
    const int n = pool.num_gs;
    uint32_t *flag = scratch;
    uint32_t *pos = scratch + n + 1;
    launch_mature_count(s, pool, st, flag, pos, d_count);
    launch_mature_pack(s, pool, F, st, record, flag, pos, d_count);
}

}  // namespace swgs
