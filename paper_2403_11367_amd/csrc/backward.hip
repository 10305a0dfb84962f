// Backward of the render (S1 + S5): gradients of a loss with respect to the
// Gaussians' means, scales, rotations (raw quaternions), opacities and colours,
// given the gradients of the rendered colour and depth images.
//
// Paper: Sec. III-A (Eq. 1-5) is differentiable; the map-training step of the
// paper's pipeline optimises the Gaussians through it. With w_i = alpha_i T_i,
//   C = sum_i c_i w_i,  D = sum_i z_i w_i,  T_i = prod_{j<i} (1 - alpha_j),
//   dC/dc_i = w_i,  dC/dz_i = 0,  dD/dz_i = w_i,
//   dC/dalpha_i = c_i T_i - S_i / (1 - alpha_i),  S_i = sum_{j>i} c_j w_j,
// and alpha_i = o_i exp(-d_i^2 / 2) (unless clamped at alpha_max, where it is
// constant). The contributing set (support cutoff, alpha floor, the layer after
// which the pixel stops) is piecewise constant and is taken as fixed.
//
// The compositing backward (screen-space gradients per (pose, Gaussian)) runs
// the forward's tile walk and lives with it in blend.hip. This file chains them
// to the parameters:
//
// k_project_backward: per (pose, Gaussian), the chain through the conic
// inverse, Sigma' = T Sigma T^T (Eq. 3), T = J R_w and the Jacobian of Eq. 4
// (with its clamp), the projected mean and the depth, to the mean and the six
// unique covariance entries.
//
// k_param_grads: per Gaussian, sums the poses in order and chains
// Sigma = M M^T, M = R(q) diag(s), and the quaternion normalisation.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr int kPoseGrads = 13;    // mean (3), Sigma unique entries (6), opacity, r, g, b

// Per (pose, Gaussian): screen-space gradients -> mean and covariance entries.
__global__ __launch_bounds__(kThreads) void k_project_backward(
    const float4 *__restrict__ packed, int64_t n, const float *__restrict__ poses, int n_poses, Camera cam,
    Consts kc, const uint64_t *__restrict__ vmask, const float *__restrict__ gscreen, float *__restrict__ gout) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= (int64_t)n_poses * n) return;
    const int p = (int)(idx / n);
    const int64_t g = idx - (int64_t)p * n;
    float *out = gout + idx * kPoseGrads;
    // culled in the forward (bit g % 64 of the pose's region g / 64)
    if (((vmask[(int64_t)p * ((n + 63) >> 6) + (g >> 6)] >> (g & 63)) & 1ull) == 0) {
        for (int i = 0; i < kPoseGrads; ++i) out[i] = 0.f;
        return;
    }
    const float *gs = gscreen + idx * kScreenGrads;
    const float gu = gs[0], gv = gs[1], gA = gs[2], gB = gs[3], gC = gs[4], gz = gs[9];
    const float4 q0 = packed[g * kPackedQuads], q1 = packed[g * kPackedQuads + 1], q2 = packed[g * kPackedQuads + 2];
    const float S[3][3] = {{q1.x, q1.y, q1.z}, {q1.y, q1.w, q2.x}, {q1.z, q2.x, q2.y}};
    const float *P = poses + p * 12;
    const float R[3][3] = {{P[0], P[1], P[2]}, {P[4], P[5], P[6]}, {P[8], P[9], P[10]}};
    float t[3];
    for (int i = 0; i < 3; ++i) t[i] = R[i][0] * q0.x + R[i][1] * q0.y + R[i][2] * q0.z + P[4 * i + 3];
    const float tz = t[2], iz = 1.f / tz;
    const float xt = t[0] * iz, yt = t[1] * iz;
    const float lim_x = kc.jac_clamp * ((0.5f * (float)cam.width) / cam.fx);
    const float lim_y = kc.jac_clamp * ((0.5f * (float)cam.height) / cam.fy);
    const bool free_x = xt > -lim_x && xt < lim_x, free_y = yt > -lim_y && yt < lim_y;
    const float xc = fminf(fmaxf(xt, -lim_x), lim_x), yc = fminf(fmaxf(yt, -lim_y), lim_y);
    const float J[2][3] = {{cam.fx * iz, 0.f, -cam.fx * xc * iz}, {0.f, cam.fy * iz, -cam.fy * yc * iz}};
    float T[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) T[i][j] = J[i][0] * R[0][j] + J[i][1] * R[1][j] + J[i][2] * R[2][j];
    // Sigma' = T S T^T + eps I, conic Q = Sigma'^-1 (as the forward computes it)
    float TS[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) TS[i][j] = T[i][0] * S[0][j] + T[i][1] * S[1][j] + T[i][2] * S[2][j];
    const float a = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + kc.eps;
    const float b = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
    const float c = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + kc.eps;
    const float det = a * c - b * b;
    const float A = c / det, B = -b / det, C = a / det;
    // dL/dSigma' = -Q G_Q Q with G_Q = [[gA, gB/2], [gB/2, gC]] (B appears twice in d^2)
    const float hb = 0.5f * gB;
    const float P00 = gA * A + hb * B, P01 = gA * B + hb * C, P10 = hb * A + gC * B, P11 = hb * B + gC * C;
    const float X00 = A * P00 + B * P10, X01 = A * P01 + B * P11, X11 = B * P01 + C * P11;
    // matrix gradient of the symmetric Sigma': Gs = -X
    const float Gs[2][2] = {{-X00, -X01}, {-X01, -X11}};
    // dL/dS = T^T Gs T; dL/dT = 2 Gs T S
    float GT[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) GT[i][j] = Gs[i][0] * T[0][j] + Gs[i][1] * T[1][j];
    float gS[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gS[i][j] = T[0][i] * GT[0][j] + T[1][i] * GT[1][j];
    float dT[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) dT[i][j] = 2.f * (GT[i][0] * S[0][j] + GT[i][1] * S[1][j] + GT[i][2] * S[2][j]);
    // T = J R: dL/dJ = dT R^T; only J00, J02, J11, J12 depend on t
    const float gJ00 = dT[0][0] * R[0][0] + dT[0][1] * R[0][1] + dT[0][2] * R[0][2];
    const float gJ02 = dT[0][0] * R[2][0] + dT[0][1] * R[2][1] + dT[0][2] * R[2][2];
    const float gJ11 = dT[1][0] * R[1][0] + dT[1][1] * R[1][1] + dT[1][2] * R[1][2];
    const float gJ12 = dT[1][0] * R[2][0] + dT[1][1] * R[2][1] + dT[1][2] * R[2][2];
    const float iz2 = iz * iz;
    float gtx = 0.f, gty = 0.f, gtz = gz;
    gtz -= gJ00 * cam.fx * iz2 + gJ11 * cam.fy * iz2;
    if (free_x) {  // J02 = -fx tx / tz^2
        gtx -= gJ02 * cam.fx * iz2;
        gtz += gJ02 * 2.f * cam.fx * t[0] * iz2 * iz;
    } else {       // J02 = -fx xc / tz
        gtz += gJ02 * cam.fx * xc * iz2;
    }
    if (free_y) {
        gty -= gJ12 * cam.fy * iz2;
        gtz += gJ12 * 2.f * cam.fy * t[1] * iz2 * iz;
    } else {
        gtz += gJ12 * cam.fy * yc * iz2;
    }
    // u = fx tx / tz + cx, v = fy ty / tz + cy
    gtx += gu * cam.fx * iz;
    gty += gv * cam.fy * iz;
    gtz -= (gu * cam.fx * t[0] + gv * cam.fy * t[1]) * iz2;
    // t = R mu + t_w
    for (int j = 0; j < 3; ++j) out[j] = R[0][j] * gtx + R[1][j] * gty + R[2][j] * gtz;
    // unique covariance entries (00, 01, 02, 11, 12, 22); off-diagonals appear twice
    out[3] = gS[0][0];
    out[4] = gS[0][1] + gS[1][0];
    out[5] = gS[0][2] + gS[2][0];
    out[6] = gS[1][1];
    out[7] = gS[1][2] + gS[2][1];
    out[8] = gS[2][2];
    out[9] = gs[5];
    out[10] = gs[6];
    out[11] = gs[7];
    out[12] = gs[8];
}

// Per Gaussian: sum over poses, then Sigma = M M^T with M = R(q) diag(s).
__global__ __launch_bounds__(kThreads) void k_param_grads(const float *__restrict__ gpose, int64_t n, int n_poses,
                                                          const float *__restrict__ scales,
                                                          const float *__restrict__ quats, float *__restrict__ g_means,
                                                          float *__restrict__ g_scales, float *__restrict__ g_quats,
                                                          float *__restrict__ g_opacity, float *__restrict__ g_rgb) {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= n) return;
    float acc[kPoseGrads] = {};
    for (int p = 0; p < n_poses; ++p) {
        const float *src = gpose + ((int64_t)p * n + g) * kPoseGrads;
        for (int i = 0; i < kPoseGrads; ++i) acc[i] += src[i];
    }
    for (int j = 0; j < 3; ++j) g_means[g * 3 + j] = acc[j];
    g_opacity[g] = acc[9];
    for (int j = 0; j < 3; ++j) g_rgb[g * 3 + j] = acc[10 + j];
    // matrix gradient of the symmetric Sigma from its unique-entry gradients
    const float G[3][3] = {{acc[3], 0.5f * acc[4], 0.5f * acc[5]},
                           {0.5f * acc[4], acc[6], 0.5f * acc[7]},
                           {0.5f * acc[5], 0.5f * acc[7], acc[8]}};
    const float qw0 = quats[g * 4], qx0 = quats[g * 4 + 1], qy0 = quats[g * 4 + 2], qz0 = quats[g * 4 + 3];
    const float nq = sqrtf(((qw0 * qw0 + qx0 * qx0) + qy0 * qy0) + qz0 * qz0);
    const float w = qw0 / nq, x = qx0 / nq, y = qy0 / nq, z = qz0 / nq;
    const float Rm[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                            {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                            {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
    const float s[3] = {scales[g * 3], scales[g * 3 + 1], scales[g * 3 + 2]};
    float M[3][3], dM[3][3], gR[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = Rm[i][j] * s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dM[i][j] = 2.f * (G[i][0] * M[0][j] + G[i][1] * M[1][j] + G[i][2] * M[2][j]);
    for (int j = 0; j < 3; ++j) g_scales[g * 3 + j] = dM[0][j] * Rm[0][j] + dM[1][j] * Rm[1][j] + dM[2][j] * Rm[2][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gR[i][j] = dM[i][j] * s[j];
    // R(q) for the unit quaternion (w, x, y, z)
    const float gw = 2.f * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    const float gx = 2.f * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.f * x * gR[1][1] - w * gR[1][2] +
                            z * gR[2][0] + w * gR[2][1] - 2.f * x * gR[2][2]);
    const float gy = 2.f * (-2.f * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                            w * gR[2][0] + z * gR[2][1] - 2.f * y * gR[2][2]);
    const float gz = 2.f * (-2.f * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.f * z * gR[1][1] +
                            y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    // q_hat = q / |q|: dL/dq = (g - q_hat (q_hat . g)) / |q|
    const float dot = w * gw + x * gx + y * gy + z * gz;
    g_quats[g * 4 + 0] = (gw - w * dot) / nq;
    g_quats[g * 4 + 1] = (gx - x * dot) / nq;
    g_quats[g * 4 + 2] = (gy - y * dot) / nq;
    g_quats[g * 4 + 3] = (gz - z * dot) / nq;
}

}  // namespace

int pose_grads_per_gaussian() { return kPoseGrads; }

void launch_project_backward(hipStream_t s, const float4 *packed, int64_t n, const float *poses, int n_poses,
                             const Camera &cam, const Consts &k, const uint64_t *vmask, const float *gscreen,
                             float *gpose) {
    const int64_t total = (int64_t)n_poses * n;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_project_backward, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       s, packed, n, poses, n_poses, cam, k, vmask, gscreen, gpose);
}

void launch_param_grads(hipStream_t s, const float *gpose, int64_t n, int n_poses, const float *scales,
                        const float *quats, float *g_means, float *g_scales, float *g_quats, float *g_opacity,
                        float *g_rgb) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_param_grads, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, gpose,
                       n, n_poses, scales, quats, g_means, g_scales, g_quats, g_opacity, g_rgb);
}

}  // namespace gsr
