// View-dependent colour: the real spherical harmonics of degrees 1..3
// divided by Y_00 = 1 / (2 sqrt(pi)), so the degree-0 coefficient of a
// Gaussian is its colour (Sec. II-B optimises the map's SH coefficients).
// Order l = 1..3, m = -l..l; Cartesian forms without the Condon-Shortley
// sign.  With the 2 sqrt(pi) factor folded in, the constants are
//   l = 1:  sqrt(3) (y, z, x)
//   l = 2:  sqrt(15) xy, sqrt(15) yz, sqrt(5)/2 (3z^2 - 1), sqrt(15) xz,
//           sqrt(15)/2 (x^2 - y^2)
//   l = 3:  sqrt(35/8) y (3x^2 - y^2), sqrt(105) xyz, sqrt(21/8) y (5z^2 - 1),
//           sqrt(7)/2 (5z^3 - 3z), sqrt(21/8) x (5z^2 - 1),
//           sqrt(105)/2 (x^2 - y^2) z, sqrt(35/8) x (x^2 - 3y^2).
// Every function takes the basis index k as a value that is a compile-time
// constant after loop unrolling, so the switch folds away.
#pragma once

#include "common.hpp"

namespace gsl {

constexpr int kShMaxK = 15;  // degree 3

__host__ __device__ constexpr int sh_count(int degree) { return (degree + 1) * (degree + 1) - 1; }

namespace shc {
constexpr double s3 = 1.7320508075688772, s15 = 3.872983346207417, h_s5 = 1.118033988749895,
                 h_s15 = 1.9364916731037085, a = 2.091650066335189, b = 10.246950765959598,
                 h_b = 5.123475382979799, c = 1.620185174601965, e = 1.3228756555322954;
}

__device__ __forceinline__ double sh_b(int k, double x, double y, double z)
{
    using namespace shc;
    switch (k) {
    case 0: return s3 * y;
    case 1: return s3 * z;
    case 2: return s3 * x;
    case 3: return s15 * x * y;
    case 4: return s15 * y * z;
    case 5: return h_s5 * (3.0 * z * z - 1.0);
    case 6: return s15 * x * z;
    case 7: return h_s15 * (x * x - y * y);
    case 8: return a * y * (3.0 * x * x - y * y);
    case 9: return b * x * y * z;
    case 10: return c * y * (5.0 * z * z - 1.0);
    case 11: return e * (5.0 * z * z * z - 3.0 * z);
    case 12: return c * x * (5.0 * z * z - 1.0);
    case 13: return h_b * (x * x - y * y) * z;
    default: return a * x * (x * x - 3.0 * y * y);
    }
}

// Partial derivatives of the polynomial of sh_b with respect to x, y, z.
__device__ __forceinline__ void sh_db(int k, double x, double y, double z, double &dx, double &dy, double &dz)
{
    using namespace shc;
    dx = dy = dz = 0.0;
    switch (k) {
    case 0: dy = s3; break;
    case 1: dz = s3; break;
    case 2: dx = s3; break;
    case 3: dx = s15 * y; dy = s15 * x; break;
    case 4: dy = s15 * z; dz = s15 * y; break;
    case 5: dz = 6.0 * h_s5 * z; break;
    case 6: dx = s15 * z; dz = s15 * x; break;
    case 7: dx = 2.0 * h_s15 * x; dy = -2.0 * h_s15 * y; break;
    case 8: dx = 6.0 * a * x * y; dy = a * (3.0 * x * x - 3.0 * y * y); break;
    case 9: dx = b * y * z; dy = b * x * z; dz = b * x * y; break;
    case 10: dy = c * (5.0 * z * z - 1.0); dz = 10.0 * c * y * z; break;
    case 11: dz = e * (15.0 * z * z - 3.0); break;
    case 12: dx = c * (5.0 * z * z - 1.0); dz = 10.0 * c * x * z; break;
    case 13: dx = 2.0 * h_b * x * z; dy = -2.0 * h_b * y * z; dz = h_b * (x * x - y * y); break;
    default: dx = a * (3.0 * x * x - 3.0 * y * y); dy = -6.0 * a * x * y; break;
    }
}

// Unit direction from the camera centre o = -R^T t to the world point p, and
// the distance.
__device__ __forceinline__ double view_dir(const DevCam &cam, double px, double py, double pz, double u[3])
{
    const double ox = -(cam.R[0] * (double)cam.t[0] + cam.R[3] * (double)cam.t[1] + cam.R[6] * (double)cam.t[2]);
    const double oy = -(cam.R[1] * (double)cam.t[0] + cam.R[4] * (double)cam.t[1] + cam.R[7] * (double)cam.t[2]);
    const double oz = -(cam.R[2] * (double)cam.t[0] + cam.R[5] * (double)cam.t[1] + cam.R[8] * (double)cam.t[2]);
    const double dx = px - ox, dy = py - oy, dz = pz - oz;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double ir = 1.0 / r;
    u[0] = dx * ir;
    u[1] = dy * ir;
    u[2] = dz * ir;
    return r;
}

}  // namespace gsl
