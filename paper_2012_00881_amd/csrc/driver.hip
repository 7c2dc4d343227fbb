// The time loop of WAND-PIC's Algorithm 1 around the xi-sweep: driver
// macroparticles deposit their longitudinal current on planes in xi, the
// slices of the sweep add it to j_z, every slice hands its wake to the driver
// particles whose mid-step position lies between it and the slice before, and
// after the sweep the driver is advanced in t by eqs. (25)-(26).
//
// Driver state [8][stride]: x, y, xi = t - z, p_x, p_y, p_z, q/m (units of
// e/m_e) and w (number of particles in units of n0 k_p^-3).
#include "wq_common.h"

namespace wq {
namespace {

enum { DX = 0, DY, DXI, DPX, DPY, DPZ, DQM, DW };

// Fixed-point scale of the deposit planes: integer sums are exact and
// independent of the order of the atomics, so the deposit is deterministic;
// one unit is 2^-40 (about 9e-13) of the current density.
constexpr double kFix = 1099511627776.0;  // 2^40
constexpr double kUnfix = 1.0 / kFix;

__device__ __forceinline__ void cic1(double x, double L, double h, int N, int& c, double& d) {
    const double t = (x + L) / h;
    int k = (int)floor(t);
    k = k < 0 ? 0 : (k > N - 1 ? N - 1 : k);
    c = k;
    d = t - (double)k;
}

__device__ __forceinline__ void add_fix(unsigned long long* p, double v) {
    atomicAdd(p, (unsigned long long)__double2ll_rn(v * kFix));
}

// Each particle adds -qm w v_z / (h^2 dz) with CIC weights in x, y and hat
// weights in xi to the planes xi0 + m dz (padded node layout, fixed point).
__global__ void k_driver_deposit(int64_t n, int stride, const double* __restrict__ s, int N,
                                 double L, double h, int pitch, int nz, double xi0, double dz,
                                 unsigned long long* __restrict__ planes) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double x = s[DX * stride + p], y = s[DY * stride + p], xi = s[DXI * stride + p];
    if (fabs(x) > L || fabs(y) > L) return;
    const double t = (xi - xi0) / dz;
    const int m = (int)floor(t);
    if (m < 0 || m > nz - 2) return;
    const double az = t - m;
    const double px = s[DPX * stride + p], py = s[DPY * stride + p], pz = s[DPZ * stride + p];
    const double vz = pz / sqrt(1.0 + px * px + py * py + pz * pz);
    const double q = -s[DQM * stride + p] * s[DW * stride + p] * vz / (h * h * dz);
    int a, b;
    double dx, dy;
    cic1(x, L, h, N, a, dx);
    cic1(y, L, h, N, b, dy);
    const size_t plane = (size_t)(N + 1) * pitch;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        unsigned long long* P = planes + (size_t)(m + k) * plane;
        const double wz = k ? az : 1.0 - az;
        const size_t g = (size_t)b * pitch + a;
        add_fix(P + g, q * wz * (1.0 - dx) * (1.0 - dy));
        add_fix(P + g + 1, q * wz * dx * (1.0 - dy));
        add_fix(P + g + pitch, q * wz * (1.0 - dx) * dy);
        add_fix(P + g + pitch + 1, q * wz * dx * dy);
    }
}

struct SliceWake {
    const double *gx, *gy, *Ez, *Bz, *Bx, *By;
};

// Mid-step position of a driver particle: a drift of dt/2 in (x, y, xi).
__device__ __forceinline__ void mid_step(const double* s, int64_t p, int stride, double dt,
                                         double& xh, double& yh, double& xih) {
    const double px = s[DPX * stride + p], py = s[DPY * stride + p], pz = s[DPZ * stride + p];
    const double g0 = sqrt(1.0 + px * px + py * py + pz * pz);
    xh = s[DX * stride + p] + 0.5 * dt * px / g0;
    yh = s[DY * stride + p] + 0.5 * dt * py / g0;
    xih = s[DXI * stride + p] + 0.5 * dt * (1.0 - pz / g0);
}

// The wake of the slices xi_prev = st[3] (W0) and xi_cur = st[2] (W1) at the
// driver particles whose mid-step position has xi_prev <= xi < xi_cur:
// E = (-d_x psi + B_y, -d_y psi - B_x, Ez) and B, gathered (CIC) in each slice
// and interpolated linearly in xi, into eb [6][stride].
__global__ void k_driver_gather(int64_t n, int stride, const double* __restrict__ s, double dt,
                                int N, double L, double h, int pitch, const double* __restrict__ st,
                                SliceWake W0, SliceWake W1, double* __restrict__ eb) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double xh, yh, xih;
    mid_step(s, p, stride, dt, xh, yh, xih);
    const double xlo = st[3], xhi = st[2];
    if (!(xih >= xlo && xih < xhi) || fabs(xh) > L || fabs(yh) > L) return;
    const double a = (xih - xlo) / (xhi - xlo);
    int ca, cb;
    double dx, dy;
    cic1(xh, L, h, N, ca, dx);
    cic1(yh, L, h, N, cb, dy);
    const size_t g = (size_t)cb * pitch + ca;
    auto at = [&](const double* F) {
        return F[g] * (1.0 - dx) * (1.0 - dy) + F[g + 1] * dx * (1.0 - dy) +
               F[g + pitch] * (1.0 - dx) * dy + F[g + pitch + 1] * dx * dy;
    };
    const SliceWake Ws[2] = {W0, W1};
    const double ws[2] = {1.0 - a, a};
    double E[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double Gx = at(Ws[k].gx), Gy = at(Ws[k].gy);
        const double ez = at(Ws[k].Ez), bz = at(Ws[k].Bz), bx = at(Ws[k].Bx), by = at(Ws[k].By);
        E[0] += ws[k] * (-Gx + by);
        E[1] += ws[k] * (-Gy - bx);
        E[2] += ws[k] * ez;
        B[0] += ws[k] * bx;
        B[1] += ws[k] * by;
        B[2] += ws[k] * bz;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        eb[q * stride + p] = E[q];
        eb[(3 + q) * stride + p] = B[q];
    }
}

// The laser's planes at t (A0) and t + dt (A1), [nz][N+1][pitch] complex, for
// the driver push (A0 null: no laser).
struct LaserPair {
    const double2* A0;
    const double2* A1;
    int nz;
    double dxi0, k0;
    size_t plane;
};

// The laser's high-frequency fields (Sec. IV, eqs. (21)-(24)) at (x, y, xi)
// and time t + tau dt, added to E and B.  The envelope is the interpolant
// linear in t between A0 and A1, linear in xi between the planes xi_m = m dxi0
// around xi (planes outside [0, nz) are zero) and bilinear in x, y; its
// derivatives are the interpolant's.  With e = exp(-i k0 xi):
//   E_x += Re[-(d_t A + d_xi A - i k0 A) e],  B_y += Re[(-d_xi A + i k0 A) e],
//   E_z += Re[-d_x A e],                      B_z += Re[-d_y A e];
// nothing outside the transverse box.
__device__ void laser_fields(const LaserPair& Lz, int N, double L, double h, int pitch, double dt,
                             double tau, double x, double y, double xi, double (&E)[3],
                             double (&B)[3]) {
    if (fabs(x) > L || fabs(y) > L) return;
    int a, b;
    double dx, dy;
    cic1(x, L, h, N, a, dx);
    cic1(y, L, h, N, b, dy);
    const double t = xi / Lz.dxi0;
    const double mf = floor(t);
    const double wz = t - mf;
    const size_t g = (size_t)b * pitch + a;
    // [time level][plane m, m + 1]: value, d/dx, d/dy of the bilinear interpolant
    double2 v[2][2], vx[2][2], vy[2][2];
    const double2* As[2] = {Lz.A0, Lz.A1};
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double q = mf + k;
            v[l][k] = vx[l][k] = vy[l][k] = make_double2(0.0, 0.0);
            if (q < 0.0 || q >= Lz.nz) continue;
            const double2* P = As[l] + (size_t)q * Lz.plane + g;
            const double2 f00 = P[0], f10 = P[1], f01 = P[pitch], f11 = P[pitch + 1];
            const double w00 = (1.0 - dx) * (1.0 - dy), w10 = dx * (1.0 - dy), w01 = (1.0 - dx) * dy,
                         w11 = dx * dy;
            v[l][k] = make_double2(f00.x * w00 + f10.x * w10 + f01.x * w01 + f11.x * w11,
                                   f00.y * w00 + f10.y * w10 + f01.y * w01 + f11.y * w11);
            vx[l][k] = make_double2(((f10.x - f00.x) * (1.0 - dy) + (f11.x - f01.x) * dy) / h,
                                    ((f10.y - f00.y) * (1.0 - dy) + (f11.y - f01.y) * dy) / h);
            vy[l][k] = make_double2(((f01.x - f00.x) * (1.0 - dx) + (f11.x - f10.x) * dx) / h,
                                    ((f01.y - f00.y) * (1.0 - dx) + (f11.y - f10.y) * dx) / h);
        }
    const double wt[2] = {1.0 - tau, tau}, wq[2] = {1.0 - wz, wz};
    double2 A = make_double2(0.0, 0.0), At = A, Axi = A, Ax = A, Ay = A;
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double w = wt[l] * wq[k];
            A.x += w * v[l][k].x;
            A.y += w * v[l][k].y;
            Ax.x += w * vx[l][k].x;
            Ax.y += w * vx[l][k].y;
            Ay.x += w * vy[l][k].x;
            Ay.y += w * vy[l][k].y;
        }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        At.x += wq[k] * (v[1][k].x - v[0][k].x) / dt;
        At.y += wq[k] * (v[1][k].y - v[0][k].y) / dt;
    }
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        Axi.x += wt[l] * (v[l][1].x - v[l][0].x) / Lz.dxi0;
        Axi.y += wt[l] * (v[l][1].y - v[l][0].y) / Lz.dxi0;
    }
    const double c = cos(Lz.k0 * xi), sn = -sin(Lz.k0 * xi);  // e = c + i sn
    // i k0 A
    const double ikx = -Lz.k0 * A.y, iky = Lz.k0 * A.x;
    auto re = [&](double zr, double zi) { return zr * c - zi * sn; };  // Re[z e]
    E[0] += re(-(At.x + Axi.x - ikx), -(At.y + Axi.y - iky));
    E[2] += re(-Ax.x, -Ax.y);
    B[1] += re(ikx - Axi.x, iky - Axi.y);
    B[2] += re(-Ay.x, -Ay.y);
}

// One step dt of eqs. (25)-(26) in nsub sub-steps (the sub-cycling of Sec. IV
// that resolves the laser's oscillation).  Each sub-step of length d: drift
// d/2, kick d/2 by qm E, the rotation of a Boris push about qm B / gamma, kick
// d/2, drift d/2 with the new momentum (a volume-preserving splitting), with
// E, B = the wake gathered at the mid-step position of the whole step (eb)
// plus, with a laser, its fields at the sub-step's mid position and time.
__global__ void k_driver_push(int64_t n, int stride, double* __restrict__ s, double dt, int nsub,
                              const double* __restrict__ eb, LaserPair las, int N, double L,
                              double h, int pitch) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double Ew[3] = {eb[p], eb[stride + p], eb[2 * stride + p]};
    const double Bw[3] = {eb[3 * stride + p], eb[4 * stride + p], eb[5 * stride + p]};
    const double qm = s[DQM * stride + p];
    double x = s[DX * stride + p], y = s[DY * stride + p], xi = s[DXI * stride + p];
    double px = s[DPX * stride + p], py = s[DPY * stride + p], pz = s[DPZ * stride + p];
    const double d = dt / nsub;
    for (int sub = 0; sub < nsub; ++sub) {
        const double g0 = sqrt(1.0 + px * px + py * py + pz * pz);
        const double xh = x + 0.5 * d * px / g0;
        const double yh = y + 0.5 * d * py / g0;
        const double xih = xi + 0.5 * d * (1.0 - pz / g0);
        double E[3] = {Ew[0], Ew[1], Ew[2]}, B[3] = {Bw[0], Bw[1], Bw[2]};
        if (las.A0) laser_fields(las, N, L, h, pitch, dt, (sub + 0.5) / nsub, xh, yh, xih, E, B);
        const double k = 0.5 * d * qm;
        const double m[3] = {px + k * E[0], py + k * E[1], pz + k * E[2]};
        const double gm = sqrt(1.0 + m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        const double t[3] = {k * B[0] / gm, k * B[1] / gm, k * B[2] / gm};
        const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        const double sv[3] = {2.0 * t[0] / (1.0 + tt), 2.0 * t[1] / (1.0 + tt), 2.0 * t[2] / (1.0 + tt)};
        const double pr[3] = {m[0] + (m[1] * t[2] - m[2] * t[1]), m[1] + (m[2] * t[0] - m[0] * t[2]),
                              m[2] + (m[0] * t[1] - m[1] * t[0])};
        const double pp[3] = {m[0] + (pr[1] * sv[2] - pr[2] * sv[1]), m[1] + (pr[2] * sv[0] - pr[0] * sv[2]),
                              m[2] + (pr[0] * sv[1] - pr[1] * sv[0])};
        px = pp[0] + k * E[0];
        py = pp[1] + k * E[1];
        pz = pp[2] + k * E[2];
        const double g1 = sqrt(1.0 + px * px + py * py + pz * pz);
        x = xh + 0.5 * d * px / g1;
        y = yh + 0.5 * d * py / g1;
        xi = xih + 0.5 * d * (1.0 - pz / g1);
    }
    s[DPX * stride + p] = px;
    s[DPY * stride + p] = py;
    s[DPZ * stride + p] = pz;
    s[DX * stride + p] = x;
    s[DY * stride + p] = y;
    s[DXI * stride + p] = xi;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

wandqs_status driver_deposit(wandqs_ctx* c) {
    const size_t words = (size_t)c->drv_nz * (c->N + 1) * c->lev[0].pitch;
    WQ_HIP(hipMemsetAsync(c->drv_planes, 0, words * sizeof(unsigned long long), c->stream));
    if (c->drv_n > 0) {
        ProfScope ps(c, "k_driver_deposit", (double)c->drv_n * 56.0);
        WQ_KLAUNCH(ps, k_driver_deposit, dim3(blocks(c->drv_n)), dim3(256), 0, c->stream, c->drv_n,
                   c->cfg.driver_max, c->drv, c->N, c->L, c->h, c->lev[0].pitch, c->drv_nz,
                   c->cfg.driver_xi0, c->cfg.driver_dz, c->drv_planes);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status driver_gather(wandqs_ctx* c, double dt) {
    if (c->drv_n <= 0) return WANDQS_OK;
    const SliceWake w0{c->gpsi_prev[0], c->gpsi_prev[1], c->fields_prev[1], c->fields_prev[2],
                       c->fields_prev[3], c->fields_prev[4]};
    const SliceWake w1{c->gpsi[0], c->gpsi[1], c->fields[1], c->fields[2], c->fields[3], c->fields[4]};
    {
        ProfScope ps(c, "k_driver_gather", (double)c->drv_n * 96.0);
        WQ_KLAUNCH(ps, k_driver_gather, dim3(blocks(c->drv_n)), dim3(256), 0, c->stream, c->drv_n,
                   c->cfg.driver_max, c->drv, dt, c->N, c->L, c->h, c->lev[0].pitch, c->st, w0, w1,
                   c->drv_eb);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status driver_push(wandqs_ctx* c, double dt) {
    if (c->drv_n <= 0) return WANDQS_OK;
    const int nsub = c->cfg.driver_nsub > 1 ? c->cfg.driver_nsub : 1;
    // the laser's planes at t and t + dt: the time step has advanced them but
    // not yet made the new set the current one
    LaserPair las{nullptr, nullptr, 0, c->cfg.dxi0, c->cfg.laser_k0,
                  (size_t)(c->N + 1) * c->lev[0].pitch};
    if (c->las_on) {
        las.A0 = c->las_env[c->las_cur];
        las.A1 = c->las_env[1 - c->las_cur];
        las.nz = c->cfg.laser_nz;
    }
    {
        ProfScope ps(c, "k_driver_push", (double)c->drv_n * 144.0);
        WQ_KLAUNCH(ps, k_driver_push, dim3(blocks(c->drv_n)), dim3(256), 0, c->stream, c->drv_n,
                   c->cfg.driver_max, c->drv, dt, nsub, c->drv_eb, las, c->N, c->L, c->h,
                   c->lev[0].pitch);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

}  // namespace wq
