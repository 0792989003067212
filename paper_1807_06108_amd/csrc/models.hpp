// Device models: explicit-Euler dynamics and state costs of the three systems,
// fp32, one sample per lane, state in registers.
//
// The paper's dynamics are the control-affine SDE of eqs. (2) and (4) with the
// noise entering through the sampled control (Algorithm 1).  The systems are
// those of Sec. VI; their equations (the paper does not print them) are:
//   double integrator: p' = v, v' = u.
//   cartpole (theta = 0 upright, uniform-rod pole of half length l):
//     tmp = (F + m_p l theta'^2 sin theta) / (m_c + m_p)
//     theta'' = (g sin theta - cos theta tmp) / (l (4/3 - m_p cos^2 theta / (m_c + m_p)))
//     p''     = tmp - m_p l theta'' cos theta / (m_c + m_p)
//   quadrotor, "+" frame, rotor thrusts f1..f4, ZYX Euler angles, body rates:
//     tau = (L (f2 - f4), L (f3 - f1), k (f1 - f2 + f3 - f4))
//     v'  = R e3 sum(f) / mass - g e3 + gust / mass
//     Euler-angle rates = W(phi, theta) omega,  omega' = J^-1 (tau - omega x J omega)
//     crash (sticky, state frozen): z < z_min or |roll| or |pitch| > tilt_max.
// Hardware transcendentals are used throughout (sine/cosine in revolutions,
// reciprocal): their error is far below the fp32 propagation error of a
// trajectory.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/mppi_jump.h"

namespace mppi {

constexpr float kInv2Pi = 0.159154943091895335769f;

__device__ __forceinline__ float fsin(float x) { return __builtin_amdgcn_sinf(x * kInv2Pi); }
__device__ __forceinline__ float fcos(float x) { return __builtin_amdgcn_cosf(x * kInv2Pi); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Host-derived constants of a model, as passed to the kernels.
struct ModelConsts {
  float c[16];
};

template <int DYN>
struct Model;

// ---------------------------------------------------------------- double integrator
template <>
struct Model<MPPI_DYN_LINEAR> {
  static constexpr int N = 2, M = 1, Q = 1;
  static constexpr int NBLK = 1, COUNT_WORD = 2;
  static constexpr bool JUMP_IN_CONTROL = true;
  static constexpr bool CAN_CRASH = false;

  __device__ __forceinline__ static void step(float* x, const float* v, const float* /*gust*/,
                                              float dt, const ModelConsts& /*mc*/) {
    const float p = x[0], vel = x[1];
    x[0] = p + vel * dt;
    x[1] = vel + v[0] * dt;
  }
  __device__ __forceinline__ static bool crashed(const float*, const ModelConsts&) {
    return false;
  }
};

// ---------------------------------------------------------------- cartpole
// consts: 0 g, 1 1/(m_c+m_p), 2 m_p l, 3 m_p l/(m_c+m_p), 4 (4/3) l
template <>
struct Model<MPPI_DYN_CARTPOLE> {
  static constexpr int N = 4, M = 1, Q = 1;
  static constexpr int NBLK = 1, COUNT_WORD = 2;
  static constexpr bool JUMP_IN_CONTROL = true;
  static constexpr bool CAN_CRASH = false;

  __device__ __forceinline__ static void step(float* x, const float* v, const float* /*gust*/,
                                              float dt, const ModelConsts& mc) {
    const float g = mc.c[0], invM = mc.c[1], mpl = mc.c[2], mplM = mc.c[3], l43 = mc.c[4];
    const float th = x[2], thd = x[3];
    const float s = fsin(th), c = fcos(th);
    const float tmp = (v[0] + mpl * thd * thd * s) * invM;
    const float thdd = (g * s - c * tmp) * frcp(l43 - mplM * c * c);
    const float pdd = tmp - mplM * thdd * c;
    x[0] = x[0] + x[1] * dt;
    x[1] = x[1] + pdd * dt;
    x[2] = th + thd * dt;
    x[3] = thd + thdd * dt;
  }
  __device__ __forceinline__ static bool crashed(const float*, const ModelConsts&) {
    return false;
  }
};

// ---------------------------------------------------------------- quadrotor
// consts: 0 1/mass, 1 1/Jx, 2 1/Jy, 3 1/Jz, 4 Jz-Jy, 5 Jx-Jz, 6 Jy-Jx,
//         7 arm, 8 k_yaw, 9 g, 10 tilt_max, 11 z_min
template <>
struct Model<MPPI_DYN_QUADROTOR> {
  static constexpr int N = 12, M = 4, Q = 3;
  // 7 normals fill two blocks; the count word takes their unused low bytes
  static constexpr int NBLK = 2, COUNT_WORD = -1;
  static constexpr bool JUMP_IN_CONTROL = false;
  static constexpr bool CAN_CRASH = true;

  __device__ __forceinline__ static void step(float* x, const float* f, const float* gust,
                                              float dt, const ModelConsts& mc) {
    const float invm = mc.c[0];
    const float L = mc.c[7], ky = mc.c[8], g = mc.c[9];
    const float phi = x[6], th = x[7], psi = x[8];
    const float p = x[9], q = x[10], r = x[11];
    const float sph = fsin(phi), cph = fcos(phi);
    const float sth = fsin(th), cth = fcos(th);
    const float sps = fsin(psi), cps = fcos(psi);
    const float thrust = (f[0] + f[1]) + (f[2] + f[3]);
    const float a = thrust * invm;
    const float ax = (cps * sth * cph + sps * sph) * a + gust[0] * invm;
    const float ay = (sps * sth * cph - cps * sph) * a + gust[1] * invm;
    const float az = (cth * cph) * a + gust[2] * invm - g;
    const float icth = frcp(cth);
    const float qr = q * sph + r * cph;
    const float phid = p + qr * sth * icth;
    const float thd = q * cph - r * sph;
    const float psid = qr * icth;
    const float tx = L * (f[1] - f[3]);
    const float ty = L * (f[2] - f[0]);
    const float tz = ky * ((f[0] - f[1]) + (f[2] - f[3]));
    const float pd = (tx - mc.c[4] * q * r) * mc.c[1];
    const float qd = (ty - mc.c[5] * r * p) * mc.c[2];
    const float rd = (tz - mc.c[6] * p * q) * mc.c[3];
    x[0] = x[0] + x[3] * dt;
    x[1] = x[1] + x[4] * dt;
    x[2] = x[2] + x[5] * dt;
    x[3] = x[3] + ax * dt;
    x[4] = x[4] + ay * dt;
    x[5] = x[5] + az * dt;
    x[6] = phi + phid * dt;
    x[7] = th + thd * dt;
    x[8] = psi + psid * dt;
    x[9] = p + pd * dt;
    x[10] = q + qd * dt;
    x[11] = r + rd * dt;
  }
  __device__ __forceinline__ static bool crashed(const float* x, const ModelConsts& mc) {
    const float tilt = mc.c[10], zmin = mc.c[11];
    return (x[2] < zmin) || (fabsf(x[6]) > tilt) || (fabsf(x[7]) > tilt);
  }
};

}  // namespace mppi
