// HIP kernels for gfx950: collocation operator, tensor-trick preconditioner,
// and the FP64 pieces of flexible GMRES.  All vectors FP64, layout
// [request][alpha][M'][z][x][y] (y fastest).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fm_internal.h"

namespace fm {

namespace {

// ---------------------------------------------------------------------------
// 1D basis helpers on the device.

__device__ __forceinline__ int dev_interval(const DimDev &d, double t) {
    int lo = 0, hi = d.K - 1;          // find the last m in [0, K-1] with nodes[m] <= t
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d.nodes[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int dev_gindex(const DimDev &d, int m, int k) {
    if (d.drop0 && k == 0 && (m == 0 || m == d.K)) return -1;
    int g = m * d.q + k - d.drop0;
    if (d.drop0 && m == d.K) g -= 1;
    return g;
}

// Values of the 2q Hermite functions nonzero at t (slot e*q + k) and their
// global indices; each carries the factor (h/hbar)^k of its derivative order.
__device__ __forceinline__ void dev_eval(const DimDev &d, double t, int *g, double *v) {
    int m = dev_interval(d, t);
    double t0 = d.nodes[m], h = d.nodes[m + 1] - t0;
    double s = (t - t0) / h, r = h / d.hbar;
    double s2 = s * s, s3 = s2 * s;
    if (d.q == 2) {
        v[0] = 1.0 - 3.0 * s2 + 2.0 * s3;
        v[1] = r * (s - 2.0 * s2 + s3);
        v[2] = 3.0 * s2 - 2.0 * s3;
        v[3] = r * (s3 - s2);
    } else {
        double s4 = s3 * s, s5 = s4 * s, r2 = r * r;
        v[0] = 1.0 - 10.0 * s3 + 15.0 * s4 - 6.0 * s5;
        v[1] = r * (s - 6.0 * s3 + 8.0 * s4 - 3.0 * s5);
        v[2] = r2 * 0.5 * (s2 - 3.0 * s3 + 3.0 * s4 - s5);
        v[3] = 10.0 * s3 - 15.0 * s4 + 6.0 * s5;
        v[4] = r * (-4.0 * s3 + 7.0 * s4 - 3.0 * s5);
        v[5] = r2 * 0.5 * (s3 - 2.0 * s4 + s5);
    }
    for (int e = 0; e < 2; ++e)
        for (int k = 0; k < d.q; ++k) g[e * d.q + k] = dev_gindex(d, m + e, k);
}

__device__ __forceinline__ bool is_cyclic(int b, int a) {
    return (b == 0 && a == 1) || (b == 1 && a == 2) || (b == 2 && a == 0);
}

// ---------------------------------------------------------------------------
// Operator: y = (H - E S) x.  One thread per spatial collocation point of one
// component; it produces all n_M outputs of that point.
__global__ void __launch_bounds__(256) k_matvec(const ProblemDev *__restrict__ pd, const double *__restrict__ Evec,
                                                const int *__restrict__ active, const double *__restrict__ X,
                                                double *__restrict__ Y) {
    const int req = blockIdx.y;
    if (active && !active[req]) return;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int a = 0;
    long long p = gid;
    while (a < 3 && p >= pd->comp[a].npts) { p -= pd->comp[a].npts; ++a; }
    if (a >= 3) return;
    const CompDev &C = pd->comp[a];
    const int nM = pd->nM, J = pd->J, M0 = pd->M0;
    const int nx = C.x.n, ny = C.y.n;
    const int iz = int(p / C.nxy), rem = int(p % C.nxy), ix = rem / ny, iy = rem % ny;
    const double *x = X + (long long)req * pd->N;
    const double E = Evec[req];
    const double zc = C.z.pts[iz], xc = C.x.pts[ix], yc = C.y.pts[iy];

    // local rows of the 1D matrices
    int gz[MAXR], gx[MAXR], gy[MAXR];
    double Sz[MAXR], D1z[MAXR], D2z[MAXR], Sx[MAXR], D2x[MAXR], Sy[MAXR], D2y[MAXR];
    const int rz = 2 * C.z.q, rx = 2 * C.x.q, ry = 2 * C.y.q;
    for (int s = 0; s < rz; ++s) {
        gz[s] = C.z.idx[iz * MAXR + s];
        Sz[s] = C.z.S[iz * MAXR + s];
        D1z[s] = C.z.D1[iz * MAXR + s];
        D2z[s] = C.z.D2[iz * MAXR + s];
    }
    for (int s = 0; s < rx; ++s) {
        gx[s] = C.x.idx[ix * MAXR + s];
        Sx[s] = C.x.S[ix * MAXR + s];
        D2x[s] = C.x.D2[ix * MAXR + s];
    }
    for (int s = 0; s < ry; ++s) {
        gy[s] = C.y.idx[iy * MAXR + s];
        Sy[s] = C.y.S[iy * MAXR + s];
        D2y[s] = C.y.D2[iy * MAXR + s];
    }

    double u[MAXM], uz[MAXM], uzz[MAXM], uxx[MAXM], uyy[MAXM];
    for (int iM = 0; iM < nM; ++iM) {
        const double *c = x + C.off + (long long)iM * C.npts;
        double s0 = 0, s1 = 0, s2 = 0, sxx = 0, syy = 0;
        for (int a1 = 0; a1 < rz; ++a1) {
            if (gz[a1] < 0) continue;
            double b00 = 0, b20 = 0, b02 = 0;
            for (int a2 = 0; a2 < rx; ++a2) {
                if (gx[a2] < 0) continue;
                const double *row = c + ((long long)gz[a1] * nx + gx[a2]) * ny;
                double t0 = 0, t2 = 0;
                for (int a3 = 0; a3 < ry; ++a3) {
                    if (gy[a3] < 0) continue;
                    double cv = row[gy[a3]];
                    t0 += Sy[a3] * cv;
                    t2 += D2y[a3] * cv;
                }
                b00 += Sx[a2] * t0;
                b20 += D2x[a2] * t0;
                b02 += Sx[a2] * t2;
            }
            s0 += Sz[a1] * b00;
            s1 += D1z[a1] * b00;
            s2 += D2z[a1] * b00;
            sxx += Sz[a1] * b20;
            syy += Sz[a1] * b02;
        }
        u[iM] = s0; uz[iM] = s1; uzz[iM] = s2; uxx[iM] = sxx; uyy[iM] = syy;
    }

    const double P = C.P[p];
    const double iy2 = 1.0 / (yc * yc), inv2 = 1.0 / (xc * xc) + iy2, omz = 1.0 - zc * zc;
    double out[MAXM];
    for (int iM = 0; iM < nM; ++iM) {
        const int Mp = M0 + iM;
        double o = -uyy[iM] - uxx[iM] -
                   inv2 * (omz * uzz[iM] - 2.0 * (Mp + 1) * zc * uz[iM] - double(Mp) * (Mp + 1) * u[iM]) +
                   ((double(J) * (J + 1) - 2.0 * Mp * Mp) * iy2 + P - E) * u[iM];
        if (iM + 1 < nM) o += pd->lhp[iM] * iy2 * (-omz * uz[iM + 1] + 2.0 * (Mp + 1) * zc * u[iM + 1]);
        if (iM > 0) o += pd->lhm[iM] * iy2 * uz[iM - 1];
        out[iM] = o;
    }

    // coupling to the other two components at the rotated points
    const double vs = C.Vs[ix * ny + iy];
    if (vs != 0.0) {
        for (int b = 0; b < 3; ++b) {
            if (b == a) continue;
            const CompDev &B = pd->comp[b];
            const double c = C.c[b], s = C.s[b];
            double xb = sqrt(fmax(c * c * xc * xc + 2.0 * s * c * xc * yc * zc + s * s * yc * yc, 0.0));
            double yb = sqrt(fmax(s * s * xc * xc - 2.0 * s * c * xc * yc * zc + c * c * yc * yc, 0.0));
            if (!(xb <= B.x.R && yb <= B.y.R)) continue;
            double den = xb * yb;
            double zb = den > 0.0 ? (s * c * (yc * yc - xc * xc) + (c * c - s * s) * xc * yc * zc) / den : 0.0;
            zb = fmin(1.0, fmax(-1.0, zb));
            int hz[MAXR], hx[MAXR], hy[MAXR];
            double vz[MAXR], vx[MAXR], vy[MAXR];
            dev_eval(B.z, zb, hz, vz);
            dev_eval(B.x, xb, hx, vx);
            dev_eval(B.y, yb, hy, vy);
            const int bnx = B.x.n, bny = B.y.n;
            const int bz_r = 2 * B.z.q, bx_r = 2 * B.x.q, by_r = 2 * B.y.q;
            double val[MAXM];
            for (int iM = 0; iM < nM; ++iM) {
                const double *cb = x + B.off + (long long)iM * B.npts;
                double acc = 0;
                for (int a1 = 0; a1 < bz_r; ++a1) {
                    if (hz[a1] < 0) continue;
                    double accx = 0;
                    for (int a2 = 0; a2 < bx_r; ++a2) {
                        if (hx[a2] < 0) continue;
                        const double *row = cb + ((long long)hz[a1] * bnx + hx[a2]) * bny;
                        double accy = 0;
                        for (int a3 = 0; a3 < by_r; ++a3)
                            if (hy[a3] >= 0) accy += vy[a3] * row[hy[a3]];
                        accx += vx[a2] * accy;
                    }
                    acc += vz[a1] * accx;
                }
                val[iM] = acc;
            }
            const double base = vs * xc * yc / den;
            if (J == 0) {
                out[0] += base * val[0];
            } else {
                double arg = (-s * xc * zc + c * yc) / yb;
                arg = fmin(1.0, fmax(-1.0, arg));
                double cw = sqrt(0.5 * (1.0 + arg)), sw = sqrt(0.5 * (1.0 - arg));
                if (!is_cyclic(b, a)) cw = -cw;
                double sa = sqrt(fmax(omz, 0.0)), sb = sqrt(fmax(1.0 - zb * zb, 0.0));
                double cpow[2 * MAXM + 2], spow[2 * MAXM + 2];
                cpow[0] = spow[0] = 1.0;
                for (int k = 1; k <= 2 * J; ++k) { cpow[k] = cpow[k - 1] * cw; spow[k] = spow[k - 1] * sw; }
                double sbp[MAXM + 1], sap[MAXM + 1];
                sbp[0] = sap[0] = 1.0;
                for (int k = 1; k <= J; ++k) { sbp[k] = sbp[k - 1] * sb; sap[k] = sap[k - 1] * sa; }
                for (int iM = 0; iM < nM; ++iM) {
                    double acc = 0;
                    for (int jM = 0; jM < nM; ++jM) {
                        const double *G = pd->dcoef + (iM * nM + jM) * pd->dlen;
                        double f = 0;
                        for (int k = 0; k <= 2 * J; ++k) f += G[k] * cpow[k] * spow[2 * J - k];
                        acc += f * sbp[M0 + jM] * val[jM];
                    }
                    out[iM] += base * acc / sap[M0 + iM];
                }
            }
        }
    }
    double *y = Y + (long long)req * pd->N + C.off + p;
    for (int iM = 0; iM < nM; ++iM) y[(long long)iM * C.npts] = out[iM];
}

// ---------------------------------------------------------------------------
// Operator, tiled: one block per (request, component, z point, XT consecutive
// x points); threads cover the tile's (x, y) points.  The coefficients of the
// tile's local stencil are read once per M' block and contracted with the
// block's z row on the way into LDS (three planes over x support x all y).
// The coupling comes from the two-slot buffer that the coupling kernel filled
// before.  Q*: spline orders (2 cubic, 3 quintic); NM: number of M' blocks.
// n_M = 1: one thread per (x group, y point).  A block covers one z point, so
// the coefficients are contracted with that point's z row (value, first and
// second derivative) as they are read: LDS holds three planes over (x support
// of the block's groups) x (all y) instead of the z support's rows, and the
// points of an x group, which share their x support, form each row's y
// contractions once for all of the group's points (<= 4).
// Block: (component, z point, gt consecutive x groups); LDS holds the three
// planes and the x rows of the block's points.
constexpr int XG_MAX = 4;

// XCD-aware tile order of the operator kernels: a launch's blocks go to the
// 8 XCDs in turn, and the grid's x extent is a multiple of 8 (the host pads
// it), so block x of every request runs on XCD x % 8.  Block x takes tile
// (x % 8) * (gridDim.x / 8) + x / 8: each XCD works through one contiguous
// range of a request's tiles (neighbouring z points, which re-read most of
// the same coefficient rows, meet in its L2), and every request still spreads
// over all XCDs (few active requests keep the chip busy).  Tiles past the
// request's count return.
__device__ __forceinline__ int xcd_tile(int x, int padded) { return (x % 8) * (padded / 8) + x / 8; }

template <int QX, int QY, int QZ>
__global__ void __launch_bounds__(256) k_local_grouped(const ProblemDev *__restrict__ pd,
                                                       const double *__restrict__ Evec,
                                                       const int *__restrict__ active,
                                                       const double *__restrict__ X, double *__restrict__ Y,
                                                       const double *__restrict__ cbuf) {
    constexpr int RX = 2 * QX, RY = 2 * QY, RZ = 2 * QZ;
    const int req = blockIdx.y, tile = xcd_tile(blockIdx.x, gridDim.x);
    if (active && !active[req]) return;
    if (tile >= pd->comp[0].ntiles_g + pd->comp[1].ntiles_g + pd->comp[2].ntiles_g) return;
    extern __shared__ double sm[];
    // the tile's record (block-uniform): everything the coefficient reads
    // depend on, in one read
    const int *rec = pd->gtile + (size_t)tile * GT_REC;
    const int a = __builtin_amdgcn_readfirstlane(rec[GT_A]), iz = __builtin_amdgcn_readfirstlane(rec[GT_IZ]);
    const int g0 = __builtin_amdgcn_readfirstlane(rec[GT_G0]), ngt = __builtin_amdgcn_readfirstlane(rec[GT_NGT]);
    const int ixs = __builtin_amdgcn_readfirstlane(rec[GT_IXS]), ixe = __builtin_amdgcn_readfirstlane(rec[GT_IXE]);
    const int kxlo = __builtin_amdgcn_readfirstlane(rec[GT_KXLO]), kxhi = __builtin_amdgcn_readfirstlane(rec[GT_KXHI]);
    const CompDev &C = pd->comp[a];
    const int ny = C.y.n;
    const int plane_n = (kxhi - kxlo + 1) * ny;
    double *pl = sm;     // the three planes interleaved: pl[3 e + c]
    double *xS = pl + 3 * plane_n, *xD = xS + (ixe - ixs) * RX;
    const bool has = threadIdx.x < ngt * ny;
    const int gl = has ? threadIdx.x / ny : 0, iy = has ? threadIdx.x % ny : 0;
    const int px0 = C.xg[g0 + gl], pn = C.xg[g0 + gl + 1] - px0;
    const double *x = X + (long long)req * pd->N + C.off;
    // this thread's rows, read now so that they arrive with the coefficients
    int lx[RX], ly[RY];
    double Sy[RY], D2y[RY];
#pragma unroll
    for (int s = 0; s < RX; ++s) {
        const int g = C.x.idx[px0 * MAXR + s];
        lx[s] = 3 * (g >= 0 ? g - kxlo : 0) * ny;
    }
#pragma unroll
    for (int s = 0; s < RY; ++s) {
        const int g = C.y.idx[iy * MAXR + s];
        ly[s] = 3 * (g >= 0 ? g : 0);
        Sy[s] = C.y.S[iy * MAXR + s];
        D2y[s] = C.y.D2[iy * MAXR + s];
    }

    // the x rows of the tile's points, requested now and written to LDS after
    // the planes (through global-memory pointers: a flat load may alias LDS, so
    // each would wait before the next LDS write)
    typedef const __attribute__((address_space(1))) double gdouble;
    gdouble *gxS = (gdouble *)C.x.S, *gxD = (gdouble *)C.x.D2;
    const int nxr = (ixe - ixs) * RX;
    double xr[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int pp = e / RX, sx = e % RX;
        xr[u][0] = e < nxr ? gxS[(ixs + pp) * MAXR + sx] : 0.0;
        xr[u][1] = e < nxr ? gxD[(ixs + pp) * MAXR + sx] : 0.0;
    }
    {
        // the block's z row; a dropped function (value 0 in all three rows)
        // reads plane 0, which exists
        const int *zidx = C.z.idx + iz * MAXR;
        const double *zS = C.z.S + iz * MAXR, *zD1 = C.z.D1 + iz * MAXR, *zD2 = C.z.D2 + iz * MAXR;
        long long zo[RZ];
        double w0[RZ], w1[RZ], w2[RZ];
#pragma unroll
        for (int a1 = 0; a1 < RZ; ++a1) {
            const int g = zidx[a1];
            zo[a1] = (long long)(g >= 0 ? g : 0) * C.nxy;
            w0[a1] = zS[a1];
            w1[a1] = zD1[a1];
            w2[a1] = zD2[a1];
        }
        // the rows kxlo..kxhi are consecutive, so a plane is one contiguous run
        // of every z row
        const double *xb = x + (long long)kxlo * ny;
        for (int e = threadIdx.x; e < plane_n; e += 256) {
            double v[RZ];
#pragma unroll
            for (int a1 = 0; a1 < RZ; ++a1) v[a1] = xb[zo[a1] + e];
            double c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
            for (int a1 = 0; a1 < RZ; ++a1) {
                c0 += w0[a1] * v[a1];
                c1 += w1[a1] * v[a1];
                c2 += w2[a1] * v[a1];
            }
            pl[3 * e] = c0;
            pl[3 * e + 1] = c1;
            pl[3 * e + 2] = c2;
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = threadIdx.x + 256 * u;
        if (e < nxr) {
            xS[e] = xr[u][0];
            xD[e] = xr[u][1];
        }
    }
    for (int e = threadIdx.x + 512; e < nxr; e += 256) {
        const int pp = e / RX, sx = e % RX;
        xS[e] = gxS[(ixs + pp) * MAXR + sx];
        xD[e] = gxD[(ixs + pp) * MAXR + sx];
    }
    __syncthreads();
    if (!has) return;
    const double *gS = xS + (px0 - ixs) * RX, *gD = xD + (px0 - ixs) * RX;
    // s0, s1, s2: value / z / zz derivative, sxx, syy: second x / y derivative
    double s0[XG_MAX], s1[XG_MAX], s2[XG_MAX], sxx[XG_MAX], syy[XG_MAX];
#pragma unroll
    for (int q = 0; q < XG_MAX; ++q) s0[q] = s1[q] = s2[q] = sxx[q] = syy[q] = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < RX; ++a2) {
        double t00 = 0, t02 = 0, t10 = 0, t20 = 0;
#pragma unroll
        for (int a3 = 0; a3 < RY; ++a3) {
            const double *v = pl + lx[a2] + ly[a3];
            t00 += Sy[a3] * v[0];
            t02 += D2y[a3] * v[0];
            t10 += Sy[a3] * v[1];
            t20 += Sy[a3] * v[2];
        }
#pragma unroll
        for (int q = 0; q < XG_MAX; ++q)
            if (q < pn) {
                const double sx = gS[q * RX + a2], dx = gD[q * RX + a2];
                s0[q] += sx * t00;
                s1[q] += sx * t10;
                s2[q] += sx * t20;
                sxx[q] += dx * t00;
                syy[q] += sx * t02;
            }
    }
    const double E = Evec[req];
    const double zc = C.z.pts[iz], yc = C.y.pts[iy];
    const double iy2 = 1.0 / (yc * yc), omz = 1.0 - zc * zc;
    const int J = pd->J, Mp = pd->M0;
    const double cJ = (double(J) * (J + 1) - 2.0 * Mp * Mp) * iy2 - E;
    const double *c0 = cbuf + (long long)req * 2 * pd->N + C.off, *c1 = c0 + pd->N;
    double *y = Y + (long long)req * pd->N + C.off;
#pragma unroll
    for (int q = 0; q < XG_MAX; ++q)
        if (q < pn) {
            const int ix = px0 + q;
            const long long p = (long long)iz * C.nxy + ix * ny + iy;
            const double xc = C.x.pts[ix];
            const double inv2 = 1.0 / (xc * xc) + iy2;
            const double o = -syy[q] - sxx[q] -
                             inv2 * (omz * s2[q] - 2.0 * (Mp + 1) * zc * s1[q] - double(Mp) * (Mp + 1) * s0[q]) +
                             (cJ + C.P[p]) * s0[q];
            y[p] = o + c0[p] + c1[p];
        }
}

template <int QX, int QY, int QZ, int NM>
__global__ void __launch_bounds__(256) k_local_tiled(const ProblemDev *__restrict__ pd, const double *__restrict__ Evec,
                                                      const int *__restrict__ active, const double *__restrict__ X,
                                                      double *__restrict__ Y, const double *__restrict__ cbuf,
                                                      int nb) {
    constexpr int RX = 2 * QX, RY = 2 * QY, RZ = 2 * QZ;
    const int req = blockIdx.y;
    if (active && !active[req]) return;
    extern __shared__ double sm[];
    int t = xcd_tile(blockIdx.x, gridDim.x), a = 0;
    while (a < 3 && t >= pd->comp[a].ntiles) { t -= pd->comp[a].ntiles; ++a; }
    if (a >= 3) return;
    const CompDev &C = pd->comp[a];
    const int ny = C.y.n, xt = C.xt;
    const int ntx = (C.x.n + xt - 1) / xt;
    const int iz = t / ntx, ix0 = (t % ntx) * xt;
    const int nxt = min(xt, C.x.n - ix0);
    const int kxlo = C.x.first[ix0], kxhi = C.x.last[ix0 + nxt - 1];
    const int plane_n = (kxhi - kxlo + 1) * ny;
    double *pl = sm;     // the three planes interleaved: pl[3 e + c]
    const bool has = threadIdx.x < nxt * ny;
    const int ixl = has ? threadIdx.x / ny : 0, iy = has ? threadIdx.x % ny : 0;
    const int ix = ix0 + ixl;
    const double *x = X + (long long)req * pd->N;
    const double E = Evec[req];
    const double zc = C.z.pts[iz], xc = C.x.pts[ix], yc = C.y.pts[iy];

    // local rows (plane-relative offsets; dropped functions have value 0)
    int lx[RX], ly[RY];
    double Sx[RX], D2x[RX], Sy[RY], D2y[RY];
#pragma unroll
    for (int s = 0; s < RX; ++s) {
        const int g = C.x.idx[ix * MAXR + s];
        lx[s] = 3 * (g >= 0 ? g - kxlo : 0) * ny;
        Sx[s] = C.x.S[ix * MAXR + s];
        D2x[s] = C.x.D2[ix * MAXR + s];
    }
#pragma unroll
    for (int s = 0; s < RY; ++s) {
        const int g = C.y.idx[iy * MAXR + s];
        ly[s] = 3 * (g >= 0 ? g : 0);
        Sy[s] = C.y.S[iy * MAXR + s];
        D2y[s] = C.y.D2[iy * MAXR + s];
    }

    // the block's z row (offsets and the three weight rows), the same for every
    // M' block: read once into LDS (published by the loop's first barrier)
    // rather than from memory again before each block's plane loads
    __shared__ long long zoff[RZ];
    __shared__ double zw[3 * RZ];
    if (threadIdx.x < RZ) {
        // through global-memory pointers, all four before the LDS writes (a flat
        // load may alias LDS and would wait before each write)
        typedef const __attribute__((address_space(1))) int gint;
        typedef const __attribute__((address_space(1))) double gdouble;
        const int a1 = threadIdx.x, zi = iz * MAXR + a1;
        const int g = ((gint *)C.z.idx)[zi];
        const double zs = ((gdouble *)C.z.S)[zi], zd1 = ((gdouble *)C.z.D1)[zi], zd2 = ((gdouble *)C.z.D2)[zi];
        zoff[a1] = (long long)(g >= 0 ? g : 0) * C.nxy;
        zw[a1] = zs;
        zw[RZ + a1] = zd1;
        zw[2 * RZ + a1] = zd2;
    }
    double u[NM], uz[NM], uzz[NM], uxx[NM], uyy[NM];
#pragma unroll
    for (int iM = 0; iM < NM; ++iM) {
        __syncthreads();
        {
            // the block's z row, contracted into three planes as the M' block is
            // read (a dropped function, value 0 in all three rows, reads plane 0)
            long long zo[RZ];
            double w0[RZ], w1[RZ], w2[RZ];
#pragma unroll
            for (int a1 = 0; a1 < RZ; ++a1) {
                zo[a1] = zoff[a1];
                w0[a1] = zw[a1];
                w1[a1] = zw[RZ + a1];
                w2[a1] = zw[2 * RZ + a1];
            }
            // rows kxlo..kxhi are consecutive: a plane is one contiguous run of each z row;
            // with four z rows two passes' loads are issued before the first wait
            // (a pass waits for its loads before its LDS writes)
            constexpr int PU = RZ <= 4 ? 2 : 1;
            const double *xb = x + C.off + (long long)iM * C.npts + (long long)kxlo * ny;
            for (int e0 = threadIdx.x; e0 < plane_n; e0 += 256 * PU) {
                double v[PU][RZ];
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    const int e = e0 + 256 * u;
#pragma unroll
                    for (int a1 = 0; a1 < RZ; ++a1) v[u][a1] = e < plane_n ? xb[zo[a1] + e] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < PU; ++u) {
                    const int e = e0 + 256 * u;
                    if (e < plane_n) {
                        double c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
                        for (int a1 = 0; a1 < RZ; ++a1) {
                            c0 += w0[a1] * v[u][a1];
                            c1 += w1[a1] * v[u][a1];
                            c2 += w2[a1] * v[u][a1];
                        }
                        pl[3 * e] = c0;
                        pl[3 * e + 1] = c1;
                        pl[3 * e + 2] = c2;
                    }
                }
            }
        }
        __syncthreads();
        double s0 = 0, s1 = 0, s2 = 0, sxx = 0, syy = 0;
#pragma unroll
        for (int a2 = 0; a2 < RX; ++a2) {
            // the row offset is taken here, so that the row's addresses are
            // formed here too (not once for all M' blocks, held in registers)
            int ro = lx[a2];
            asm volatile("" : "+v"(ro));
            double t00 = 0, t02 = 0, t10 = 0, t20 = 0;
#pragma unroll
            for (int a3 = 0; a3 < RY; ++a3) {
                const double *v = pl + ro + ly[a3];
                t00 += Sy[a3] * v[0];
                t02 += D2y[a3] * v[0];
                t10 += Sy[a3] * v[1];
                t20 += Sy[a3] * v[2];
            }
            s0 += Sx[a2] * t00;
            s1 += Sx[a2] * t10;
            s2 += Sx[a2] * t20;
            sxx += D2x[a2] * t00;
            syy += Sx[a2] * t02;
            // the row's products complete before the next row's reads issue
            // (issued all at once the reads of a block take ~220 registers)
            asm volatile("" : "+v"(s0), "+v"(s1), "+v"(s2), "+v"(sxx), "+v"(syy) : : "memory");
        }
        u[iM] = s0; uz[iM] = s1; uzz[iM] = s2; uxx[iM] = sxx; uyy[iM] = syy;
    }
    if (!has) return;

    const long long p = (long long)iz * C.nxy + ix * ny + iy;
    const double P = C.P[p];
    const double iy2 = 1.0 / (yc * yc), inv2 = 1.0 / (xc * xc) + iy2, omz = 1.0 - zc * zc;
    const int J = pd->J, M0 = pd->M0;
    double out[NM];
#pragma unroll
    for (int iM = 0; iM < NM; ++iM) {
        const int Mp = M0 + iM;
        double o = -uyy[iM] - uxx[iM] -
                   inv2 * (omz * uzz[iM] - 2.0 * (Mp + 1) * zc * uz[iM] - double(Mp) * (Mp + 1) * u[iM]) +
                   ((double(J) * (J + 1) - 2.0 * Mp * Mp) * iy2 + P - E) * u[iM];
        if (iM + 1 < NM) o += pd->lhp[iM] * iy2 * (-omz * uz[iM + 1] + 2.0 * (Mp + 1) * zc * u[iM + 1]);
        if (iM > 0) o += pd->lhm[iM] * iy2 * uz[iM - 1];
        out[iM] = o;
    }

    // plus the coupling of both partners (slot 0, then slot 1)
    const double *c0 = cbuf + (long long)req * 2 * pd->N + C.off + p, *c1 = c0 + pd->N;
    double *y = Y + (long long)req * pd->N + C.off + p;
#pragma unroll
    for (int iM = 0; iM < NM; ++iM) y[(long long)iM * C.npts] = out[iM] + c0[(long long)iM * C.npts] + c1[(long long)iM * C.npts];
}

// Operator without the coupling for more M' blocks (n_M > 3, runtime count):
// the tiling and staging of k_local_tiled, the blocks taken one after another.
// Block M''s output needs block M'+1's value and z derivative and block
// M'-1's z derivative (the M'+-1 terms), so it is completed and stored one
// block late: three blocks' sums are held at a time, whatever n_M.
template <int QX, int QY, int QZ>
__global__ void __launch_bounds__(256) k_local_many(const ProblemDev *__restrict__ pd, const double *__restrict__ Evec,
                                                     const int *__restrict__ active, const double *__restrict__ X,
                                                     double *__restrict__ Y, const double *__restrict__ cbuf) {
    constexpr int RX = 2 * QX, RY = 2 * QY, RZ = 2 * QZ;
    const int req = blockIdx.y;
    if (active && !active[req]) return;
    extern __shared__ double sm[];
    int t = xcd_tile(blockIdx.x, gridDim.x), a = 0;
    while (a < 3 && t >= pd->comp[a].ntiles) { t -= pd->comp[a].ntiles; ++a; }
    if (a >= 3) return;
    const CompDev &C = pd->comp[a];
    const int ny = C.y.n, xt = C.xt;
    const int ntx = (C.x.n + xt - 1) / xt;
    const int iz = t / ntx, ix0 = (t % ntx) * xt;
    const int nxt = min(xt, C.x.n - ix0);
    const int kxlo = C.x.first[ix0], kxhi = C.x.last[ix0 + nxt - 1];
    const int plane_n = (kxhi - kxlo + 1) * ny;
    double *pl = sm;     // the three planes interleaved: pl[3 e + c]
    const bool has = threadIdx.x < nxt * ny;
    const int ixl = has ? threadIdx.x / ny : 0, iy = has ? threadIdx.x % ny : 0;
    const int ix = ix0 + ixl;
    const double *x = X + (long long)req * pd->N;
    const double E = Evec[req];
    const double zc = C.z.pts[iz], xc = C.x.pts[ix], yc = C.y.pts[iy];

    int lx[RX], ly[RY];
    double Sx[RX], D2x[RX], Sy[RY], D2y[RY];
#pragma unroll
    for (int s = 0; s < RX; ++s) {
        const int g = C.x.idx[ix * MAXR + s];
        lx[s] = 3 * (g >= 0 ? g - kxlo : 0) * ny;
        Sx[s] = C.x.S[ix * MAXR + s];
        D2x[s] = C.x.D2[ix * MAXR + s];
    }
#pragma unroll
    for (int s = 0; s < RY; ++s) {
        const int g = C.y.idx[iy * MAXR + s];
        ly[s] = 3 * (g >= 0 ? g : 0);
        Sy[s] = C.y.S[iy * MAXR + s];
        D2y[s] = C.y.D2[iy * MAXR + s];
    }
    __shared__ long long zoff[RZ];
    __shared__ double zw[3 * RZ];
    if (threadIdx.x < RZ) {
        typedef const __attribute__((address_space(1))) int gint;
        typedef const __attribute__((address_space(1))) double gdouble;
        const int a1 = threadIdx.x, zi = iz * MAXR + a1;
        const int g = ((gint *)C.z.idx)[zi];
        const double zs = ((gdouble *)C.z.S)[zi], zd1 = ((gdouble *)C.z.D1)[zi], zd2 = ((gdouble *)C.z.D2)[zi];
        zoff[a1] = (long long)(g >= 0 ? g : 0) * C.nxy;
        zw[a1] = zs;
        zw[RZ + a1] = zd1;
        zw[2 * RZ + a1] = zd2;
    }
    const long long p = (long long)iz * C.nxy + ix * ny + iy;
    const double P = has ? C.P[p] : 0.0;
    const double iy2 = 1.0 / (yc * yc), inv2 = 1.0 / (xc * xc) + iy2, omz = 1.0 - zc * zc;
    const int J = pd->J, M0 = pd->M0, nM = pd->nM;
    const double *c0 = cbuf + (long long)req * 2 * pd->N + C.off + p, *c1 = c0 + pd->N;
    double *y = Y + (long long)req * pd->N + C.off + p;
    // sums of the previous block (its output is stored this step) and the z
    // derivative of the one before
    double pu = 0, puz = 0, puzz = 0, puxx = 0, puyy = 0, ppuz = 0;
    for (int iM = 0; iM <= nM; ++iM) {
        double s0 = 0, s1 = 0, s2 = 0, sxx = 0, syy = 0;
        if (iM < nM) {          // the same for every thread: the barriers are uniform
            __syncthreads();
            {
                long long zo[RZ];
                double w0[RZ], w1[RZ], w2[RZ];
#pragma unroll
                for (int a1 = 0; a1 < RZ; ++a1) {
                    zo[a1] = zoff[a1];
                    w0[a1] = zw[a1];
                    w1[a1] = zw[RZ + a1];
                    w2[a1] = zw[2 * RZ + a1];
                }
                constexpr int PU = RZ <= 4 ? 2 : 1;
                const double *xb = x + C.off + (long long)iM * C.npts + (long long)kxlo * ny;
                for (int e0 = threadIdx.x; e0 < plane_n; e0 += 256 * PU) {
                    double v[PU][RZ];
#pragma unroll
                    for (int u = 0; u < PU; ++u) {
                        const int e = e0 + 256 * u;
#pragma unroll
                        for (int a1 = 0; a1 < RZ; ++a1) v[u][a1] = e < plane_n ? xb[zo[a1] + e] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < PU; ++u) {
                        const int e = e0 + 256 * u;
                        if (e < plane_n) {
                            double q0 = 0, q1 = 0, q2 = 0;
#pragma unroll
                            for (int a1 = 0; a1 < RZ; ++a1) {
                                q0 += w0[a1] * v[u][a1];
                                q1 += w1[a1] * v[u][a1];
                                q2 += w2[a1] * v[u][a1];
                            }
                            pl[3 * e] = q0;
                            pl[3 * e + 1] = q1;
                            pl[3 * e + 2] = q2;
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int a2 = 0; a2 < RX; ++a2) {
                int ro = lx[a2];
                asm volatile("" : "+v"(ro));
                double t00 = 0, t02 = 0, t10 = 0, t20 = 0;
#pragma unroll
                for (int a3 = 0; a3 < RY; ++a3) {
                    const double *v = pl + ro + ly[a3];
                    t00 += Sy[a3] * v[0];
                    t02 += D2y[a3] * v[0];
                    t10 += Sy[a3] * v[1];
                    t20 += Sy[a3] * v[2];
                }
                s0 += Sx[a2] * t00;
                s1 += Sx[a2] * t10;
                s2 += Sx[a2] * t20;
                sxx += D2x[a2] * t00;
                syy += Sx[a2] * t02;
                asm volatile("" : "+v"(s0), "+v"(s1), "+v"(s2), "+v"(sxx), "+v"(syy) : : "memory");
            }
        }
        if (iM > 0 && has) {
            // block iM - 1, with block iM's sums (zero past the last block)
            const int jM = iM - 1, Mp = M0 + jM;
            double o = -puyy - puxx - inv2 * (omz * puzz - 2.0 * (Mp + 1) * zc * puz - double(Mp) * (Mp + 1) * pu) +
                       ((double(J) * (J + 1) - 2.0 * Mp * Mp) * iy2 + P - E) * pu;
            if (iM < nM) o += pd->lhp[jM] * iy2 * (-omz * s1 + 2.0 * (Mp + 1) * zc * s0);
            if (jM > 0) o += pd->lhm[jM] * iy2 * ppuz;
            const long long q = (long long)jM * C.npts;
            y[q] = o + c0[q] + c1[q];
        }
        ppuz = puz;
        pu = s0; puz = s1; puzz = s2; puxx = sxx; puyy = syy;
    }
}

// Hermite values at s in [0, 1] of the 2Q functions of one cell of width h,
// r = h / hbar (each function carries (h/hbar)^k of its derivative order k).
template <int Q>
__device__ __forceinline__ void hermite_cell(double s, double r, double *v) {
    const double s2 = s * s, s3 = s2 * s;
    if (Q == 2) {
        v[0] = 1.0 - 3.0 * s2 + 2.0 * s3;
        v[1] = r * (s - 2.0 * s2 + s3);
        v[2] = 3.0 * s2 - 2.0 * s3;
        v[3] = r * (s3 - s2);
    } else {
        const double s4 = s3 * s, s5 = s4 * s, r2 = r * r;
        v[0] = 1.0 - 10.0 * s3 + 15.0 * s4 - 6.0 * s5;
        v[1] = r * (s - 6.0 * s3 + 8.0 * s4 - 3.0 * s5);
        v[2] = r2 * 0.5 * (s2 - 3.0 * s3 + 3.0 * s4 - s5);
        v[3] = 10.0 * s3 - 15.0 * s4 + 6.0 * s5;
        v[4] = r * (-4.0 * s3 + 7.0 * s4 - 3.0 * s5);
        v[5] = r2 * 0.5 * (s3 - 2.0 * s4 + s5);
    }
}

// Orders the LDS accesses of one wave before and after this point (the
// wave's lanes run together; only the compiler and the memory model need
// telling).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int CPL_WAVES = 4;         // waves per block of the coupling kernel
constexpr int CPL_REQ = 16;          // requests per block (grid y covers the rest)

// Coupling term of the operator for the pairs of (beta, cell) tasks.  With one
// M'' block a wave may take two tasks (neighbouring cells, from a host-built
// job list), one per half: P = 2, each lane up to two of its cell's pairs
// (pairs l and l + 32 of the task), so that each staged coefficient feeds two
// products (chosen when the tasks average more than 40 pairs); P = 1, two tasks
// of at most 32 pairs, one pair per lane.  Otherwise one task per wave, one
// pair per lane.  The wave stages
// each cell's (2QZ x 2QXY x 2QXY) coefficients of every M'' block of one
// request in LDS (zero for dropped functions), then each lane evaluates beta's
// expansion at its pairs' images by the separable sum
// sum_c v_z[c] sum_a v_x[a] sum_b v_y[b] coef[c][a][b] (LDS reads are the same
// for all lanes of a cell) and writes F val to cbuf[request][slot][alpha point].
// The basis values and factors of a pair stay in registers over the requests.
template <int QXY, int QZ, int NM, int P>
__global__ void __launch_bounds__(64 * CPL_WAVES) k_coupling_cells(const ProblemDev *__restrict__ pd,
                                                                   const int *__restrict__ active, int nb,
                                                                   const double *__restrict__ X,
                                                                   double *__restrict__ cbuf) {
    static_assert(P == 1 || NM == 1, "two pairs per lane only with one M'' block");
    constexpr int RXY = 2 * QXY, RZ = 2 * QZ, TS = RZ * RXY * RXY;
    constexpr int HALVES = NM == 1 ? 2 : 1;            // cells a wave may hold
    __shared__ __align__(16) double tile[CPL_WAVES][HALVES][NM * TS];
    __shared__ int fidx[CPL_WAVES][HALVES][RZ + 2 * RXY];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const CouplingDev &cp = pd->cpl;
    // XCD-aware order: consecutive jobs (neighbouring cells) on one XCD's L2
    const int nblk = gridDim.x, xcd = blockIdx.x % 8, per = (nblk + 7) / 8;
    const int full = nblk % 8 == 0 ? 8 : nblk % 8;     // XCDs that get `per` blocks
    const int bid = xcd < full ? xcd * per + blockIdx.x / 8 : full * per + (xcd - full) * (per - 1) + blockIdx.x / 8;
    const int job = __builtin_amdgcn_readfirstlane(bid * CPL_WAVES + wave);
    if (job >= cp.njobs) return;                       // the whole wave (no block barriers)
    // the lane's task record, found from the job index alone (with two halves,
    // the job-ordered record of the lane's half; with one, job j is task j): the
    // cell's function indices and beta's sizes come with it, so the fetch of the
    // cell's coefficients and the pairs' data wait for this one read only
    const int *t = HALVES == 2 ? cp.jrec + (2 * (size_t)job + (lane >> 5)) * CPL_TASK
                               : cp.task + (size_t)job * CPL_TASK;
    // two cells (one per half) with two pairs per lane always, with one pair per
    // lane when the job holds a second task; else one cell over the wave (both
    // halves then read the same record)
    const bool split = HALVES == 2 && (P == 2 || __builtin_amdgcn_readfirstlane(t[CT_SPLIT]) != 0);
    const int W = split ? 32 : 64;                     // lanes per cell
    const int half = split ? lane >> 5 : 0, li = split ? lane & 31 : lane;
    const int count = t[CT_COUNT];                     // 0: this half has no task
    const bool has = count > 0;
    const int task = t[CT_TASK];
    const long long first = t[CT_FIRST];
    const int bnx = t[CT_NX], bny = t[CT_NY], bnpts = t[CT_NPTS];
    const long long boff = (long long)(((unsigned long long)(unsigned)t[CT_OFF_HI] << 32) | (unsigned)t[CT_OFF_LO]);
    if (li < RZ + 2 * RXY) fidx[wave][half][li] = t[CT_FIDX + li];
    bool mine[P];
    double vz[P][RZ], vx[P][RXY], vy[P][RXY], F[P][NM * NM];
    int outp[P], slot[P], npa[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const long long pr = first + li + W * p;
        mine[p] = li + W * p < count;
        outp[p] = slot[p] = npa[p] = 0;
        if (mine[p]) {
            hermite_cell<QZ>(cp.s[pr], cp.r[3 * (size_t)task], vz[p]);
            hermite_cell<QXY>(cp.s[cp.npairs + pr], cp.r[3 * (size_t)task + 1], vx[p]);
            hermite_cell<QXY>(cp.s[2 * cp.npairs + pr], cp.r[3 * (size_t)task + 2], vy[p]);
#pragma unroll
            for (int f = 0; f < NM * NM; ++f) F[p][f] = cp.F[(size_t)f * cp.npairs + pr];
            const int o = cp.out[pr];
            outp[p] = o >> 1;
            slot[p] = o & 1;
            // the point's own component, from its offset (an exchange-reduced
            // problem reads partner 2 from component 1, so beta alone does not fix it)
            const int a = outp[p] >= pd->comp[2].off ? 2 : (outp[p] >= pd->comp[1].off ? 1 : 0);
            npa[p] = pd->comp[a].npts;
        } else {
#pragma unroll
            for (int u = 0; u < RZ; ++u) vz[p][u] = 0.0;
#pragma unroll
            for (int u = 0; u < RXY; ++u) vx[p][u] = vy[p][u] = 0.0;
#pragma unroll
            for (int f = 0; f < NM * NM; ++f) F[p][f] = 0.0;
        }
    }
    const long long N = pd->N;
    const int r0 = blockIdx.y * CPL_REQ, r1 = min(nb, r0 + CPL_REQ);
    // this lane's tile entries (e = li + W q): offsets into beta's block of one
    // request, -1 for a dropped function, past the tile or without a task;
    // worked out once for all requests
    constexpr int EPL = HALVES == 2 ? (NM * TS + 31) / 32 : (NM * TS + 63) / 64;
    int goff[EPL];
    wave_sync();                                       // fidx written
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
        const int e = li + W * q;
        goff[q] = -1;
        if (has && e < NM * TS) {
            const int iM = e / TS, rem = e - iM * TS;
            const int c = rem / (RXY * RXY), a = (rem / RXY) % RXY, bq = rem % RXY;
            const int gz = fidx[wave][half][c], gx = fidx[wave][half][RZ + a], gy = fidx[wave][half][RZ + RXY + bq];
            if (gz >= 0 && gx >= 0 && gy >= 0) goff[q] = iM * bnpts + (gz * bnx + gx) * bny + gy;
        }
    }
    // Each wave works on its own tile, so waves synchronise only with
    // themselves; the tile of the next active request is fetched into
    // registers while the current one is evaluated.
    auto next_active = [&](int r) {
        while (r < r1 && active && !active[r]) ++r;
        return r;
    };
    double pf[EPL];
    auto fetch = [&](int r) {
        const double *x = X + (long long)r * N + boff;
#pragma unroll
        for (int q = 0; q < EPL; ++q) pf[q] = goff[q] >= 0 ? x[goff[q]] : 0.0;
    };
    int req = next_active(r0);
    if (req >= r1) return;
    fetch(req);
    while (req < r1) {
        const int nxt = next_active(req + 1);
        wave_sync();                                   // the previous tile is read
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            const int e = li + W * q;
            if (e < NM * TS) tile[wave][half][e] = pf[q];
        }
        wave_sync();                                   // this tile is written
        if (nxt < r1) fetch(nxt);
        if (mine[0]) {
            double val[P][NM];
#pragma unroll
            for (int iM = 0; iM < NM; ++iM) {
                const double *T = tile[wave][half] + iM * TS;
                double acc[P];
#pragma unroll
                for (int p = 0; p < P; ++p) acc[p] = 0;
#pragma unroll
                for (int c = 0; c < RZ; ++c) {
                    double accx[P];
#pragma unroll
                    for (int p = 0; p < P; ++p) accx[p] = 0;
#pragma unroll
                    for (int a = 0; a < RXY; ++a) {
                        const double *row = T + (c * RXY + a) * RXY;
                        double accy[P];
#pragma unroll
                        for (int p = 0; p < P; ++p) accy[p] = 0;
#pragma unroll
                        for (int bq = 0; bq < RXY; ++bq) {
                            const double cf = row[bq];
#pragma unroll
                            for (int p = 0; p < P; ++p) accy[p] += vy[p][bq] * cf;
                        }
#pragma unroll
                        for (int p = 0; p < P; ++p) accx[p] += vx[p][a] * accy[p];
                        // the row's products complete before the next row's reads
                        // issue (all of a tile's reads at once exhaust the registers)
                        if (P == 2) asm volatile("" : "+v"(accx[0]), "+v"(accx[P - 1]) : : "memory");
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) acc[p] += vz[p][c] * accx[p];
                }
#pragma unroll
                for (int p = 0; p < P; ++p) val[p][iM] = acc[p];
            }
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (mine[p]) {
                    double *y = cbuf + ((long long)req * 2 + slot[p]) * N + outp[p];
#pragma unroll
                    for (int iM = 0; iM < NM; ++iM) {
                        double o = 0;
#pragma unroll
                        for (int jM = 0; jM < NM; ++jM) o += F[p][iM * NM + jM] * val[p][jM];
                        y[(long long)iM * npa[p]] = o;
                    }
                }
        }
        req = nxt;
    }
}

// Coupling term for more M'' blocks (n_M > 3, runtime count up to MAXM): one
// wave per (beta, cell) task, one pair per lane.  For each request the wave
// stages one M'' block of the cell's coefficients at a time in LDS (the next
// block, or the next running request's first, is fetched into registers while
// the current one is evaluated), evaluates beta's expansion of that block at
// every lane's image by the separable sum, and adds it times the pair's factor
// column of that block to the lane's n_M outputs.  The factors (n_M x n_M per
// pair, column by column) are read from memory for each request.
template <int QXY, int QZ>
__global__ void __launch_bounds__(64 * CPL_WAVES) k_coupling_many(const ProblemDev *__restrict__ pd,
                                                                  const int *__restrict__ active, int nb,
                                                                  const double *__restrict__ X,
                                                                  double *__restrict__ cbuf) {
    constexpr int RXY = 2 * QXY, RZ = 2 * QZ, TS = RZ * RXY * RXY;
    constexpr int EPL = (TS + 63) / 64;
    __shared__ __align__(16) double tile[CPL_WAVES][TS];
    __shared__ int fidx[CPL_WAVES][RZ + 2 * RXY];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const CouplingDev &cp = pd->cpl;
    const int nblk = gridDim.x, xcd = blockIdx.x % 8, per = (nblk + 7) / 8;
    const int full = nblk % 8 == 0 ? 8 : nblk % 8;
    const int bid = xcd < full ? xcd * per + blockIdx.x / 8 : full * per + (xcd - full) * (per - 1) + blockIdx.x / 8;
    const int job = __builtin_amdgcn_readfirstlane(bid * CPL_WAVES + wave);
    if (job >= cp.njobs) return;                       // the whole wave (no block barriers)
    const int task = job;                              // with several M'' blocks job j is task j
    const int *t = cp.task + (size_t)task * CPL_TASK;
    const int count = t[CT_COUNT];
    const long long first = t[CT_FIRST];
    const int bnx = t[CT_NX], bny = t[CT_NY], bnpts = t[CT_NPTS];
    const long long boff = (long long)(((unsigned long long)(unsigned)t[CT_OFF_HI] << 32) | (unsigned)t[CT_OFF_LO]);
    if (lane < RZ + 2 * RXY) fidx[wave][lane] = t[CT_FIDX + lane];
    const int nM = pd->nM;
    const long long np = cp.npairs;
    const long long pr = first + lane;
    const bool mine = lane < count;
    double vz[RZ], vx[RXY], vy[RXY];
    int outp = 0, slot = 0, npa = 0;
    if (mine) {
        hermite_cell<QZ>(cp.s[pr], cp.r[3 * (size_t)task], vz);
        hermite_cell<QXY>(cp.s[np + pr], cp.r[3 * (size_t)task + 1], vx);
        hermite_cell<QXY>(cp.s[2 * np + pr], cp.r[3 * (size_t)task + 2], vy);
        const int o = cp.out[pr];
        outp = o >> 1;
        slot = o & 1;
        const int a = outp >= pd->comp[2].off ? 2 : (outp >= pd->comp[1].off ? 1 : 0);
        npa = pd->comp[a].npts;
    } else {
#pragma unroll
        for (int u = 0; u < RZ; ++u) vz[u] = 0.0;
#pragma unroll
        for (int u = 0; u < RXY; ++u) vx[u] = vy[u] = 0.0;
    }
    const long long N = pd->N;
    const int r0 = blockIdx.y * CPL_REQ, r1 = min(nb, r0 + CPL_REQ);
    int goff[EPL];
    wave_sync();                                       // fidx written
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
        const int e = lane + 64 * q;
        goff[q] = -1;
        if (e < TS) {
            const int c = e / (RXY * RXY), a = (e / RXY) % RXY, bq = e % RXY;
            const int gz = fidx[wave][c], gx = fidx[wave][RZ + a], gy = fidx[wave][RZ + RXY + bq];
            if (gz >= 0 && gx >= 0 && gy >= 0) goff[q] = (gz * bnx + gx) * bny + gy;
        }
    }
    auto next_active = [&](int r) {
        while (r < r1 && active && !active[r]) ++r;
        return r;
    };
    double pf[EPL];
    auto fetch = [&](int r, int jM) {
        const double *x = X + (long long)r * N + boff + (long long)jM * bnpts;
#pragma unroll
        for (int q = 0; q < EPL; ++q) pf[q] = goff[q] >= 0 ? x[goff[q]] : 0.0;
    };
    int req = next_active(r0);
    if (req >= r1) return;
    fetch(req, 0);
    double o[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) o[i] = 0.0;
    int jM = 0;
    while (req < r1) {
        // the block after this one: the next M'' block, or the next running request's first
        const int njM = jM + 1 < nM ? jM + 1 : 0;
        const int nreq = jM + 1 < nM ? req : next_active(req + 1);
        wave_sync();                                   // the previous tile is read
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            const int e = lane + 64 * q;
            if (e < TS) tile[wave][e] = pf[q];
        }
        wave_sync();                                   // this tile is written
        if (nreq < r1) fetch(nreq, njM);
        if (mine) {
            // the pair's factor column of this block, loaded before the contraction
            double f[MAXM];
#pragma unroll
            for (int i = 0; i < MAXM; ++i) f[i] = i < nM ? cp.F[(size_t)(i * nM + jM) * np + pr] : 0.0;
            const double *T = tile[wave];
            double acc = 0;
#pragma unroll
            for (int c = 0; c < RZ; ++c) {
                double accx = 0;
#pragma unroll
                for (int a = 0; a < RXY; ++a) {
                    const double *row = T + (c * RXY + a) * RXY;
                    double accy = 0;
#pragma unroll
                    for (int bq = 0; bq < RXY; ++bq) accy += vy[bq] * row[bq];
                    accx += vx[a] * accy;
                }
                acc += vz[c] * accx;
            }
#pragma unroll
            for (int i = 0; i < MAXM; ++i) o[i] += f[i] * acc;
            if (jM + 1 == nM) {
                double *y = cbuf + ((long long)req * 2 + slot) * N + outp;
#pragma unroll
                for (int i = 0; i < MAXM; ++i)
                    if (i < nM) y[(long long)i * npa] = o[i];
#pragma unroll
                for (int i = 0; i < MAXM; ++i) o[i] = 0.0;
            }
        }
        req = nreq;
        jM = njM;
    }
}

// ---------------------------------------------------------------------------
// Preconditioner, mode-z product: out[k'][p] = sum_k W[k'][k] in[k][p] for every
// (request, alpha, M') and p in [0, nx*ny).  64 columns per block staged in LDS.
constexpr int MZ_COLS = 64;

__global__ void __launch_bounds__(MZ_COLS) k_modez(const ProblemDev *__restrict__ pd, const PrecDev *__restrict__ pr, const int *__restrict__ active,
                                                   int which, const double *in, double *out) {
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    const int a = blockIdx.y / MAXM, iM = blockIdx.y % MAXM;
    if (iM >= pd->nM) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nz = C.z.n, nxy = C.nxy;
    const int col0 = blockIdx.x * MZ_COLS;
    if (col0 >= nxy) return;
    extern __shared__ double sm[];
    double *W = sm;                  // nz*nz
    double *T = sm + nz * nz;        // nz*MZ_COLS
    const double *Wg = F.Wz + ((size_t)iM * 2 + which) * nz * nz;
    for (int t = threadIdx.x; t < nz * nz; t += MZ_COLS) W[t] = Wg[t];
    const long long base = (long long)req * pd->N + C.off + (long long)iM * C.npts;
    const int col = col0 + threadIdx.x;
    const bool ok = col < nxy;
    for (int k = 0; k < nz; ++k) T[k * MZ_COLS + threadIdx.x] = ok ? in[base + (long long)k * nxy + col] : 0.0;
    __syncthreads();
    if (!ok) return;
    for (int k2 = 0; k2 < nz; ++k2) {
        double acc = 0;
        for (int k = 0; k < nz; ++k) acc += W[k2 * nz + k] * T[k * MZ_COLS + threadIdx.x];
        out[base + (long long)k2 * nxy + col] = acc;
    }
}

// Mode-z product with each (x, y) column held in registers (nz <= MAXNZ) and W
// in LDS (read by the whole wave at once): out[k'][p] = sum_k W[k'][k] in[k][p].
// A column's outputs are split over S threads of the block (S = 1, 2, 4 or 8,
// chosen so that small batches still fill the chip; each of them reads the
// whole column, the repeats from cache: sharing one read through LDS measured
// no faster), taking groups of four outputs in turn; consecutive threads take
// consecutive columns.  Grid: (columns / (256 / S), alpha x M', request); in
// and out may alias (the block reads all its columns before any thread writes).
// F32: the products in FP32 (inputs rounded to FP32, outputs widened).
constexpr int MZ2_THREADS = 256;

template <int MAXNZ, bool F32, class TI = double, class TO = double>
__global__ void __launch_bounds__(MZ2_THREADS) k_modez_reg(const ProblemDev *__restrict__ pd,
                                                           const PrecDev *__restrict__ pr,
                                                           const int *__restrict__ active, int which,
                                                           const TI *in, TO *out, int split) {
    using T = typename std::conditional<F32, float, double>::type;
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    const int nM = pd->nM;
    const int a = blockIdx.y / nM, iM = blockIdx.y % nM;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nz = C.z.n, nxy = C.nxy;
    const int cb = MZ2_THREADS / split;                // columns per block
    if ((int)blockIdx.x * cb >= nxy) return;
    __shared__ T W[(MAXNZ + 3) * MAXNZ];
    const int sub = threadIdx.x / cb;
    const int col = blockIdx.x * cb + (threadIdx.x - sub * cb);
    const bool ok = col < nxy;
    const long long base = (long long)req * pd->N + C.off + (long long)iM * C.npts + col;
    // the column as loaded (FP64 input: converted once all of it is in
    // flight, since a conversion per load would wait for each load in turn)
    using TL = typename std::conditional<std::is_same<TI, float>::value, float, double>::type;
    TL vd[MAXNZ];
#pragma unroll
    for (int k = 0; k < MAXNZ; ++k) vd[k] = (ok && k < nz) ? in[base + (long long)k * nxy] : (TL)0;
    // the factor, staged after the column loads are issued; up to nz = 32 all
    // of its loads first, then the LDS writes, so that the block waits on one
    // round trip (a loop that stores each value as it arrives waits once per pass)
    // (as global-memory pointers: loads through a generic pointer are flat
    // loads, which the compiler waits for one by one)
    const size_t wo = ((size_t)iM * 2 + which) * nz * nz;
    const int wn = (nz + 3) * nz;
    typedef const __attribute__((address_space(1))) double gdouble;
    typedef const __attribute__((address_space(1))) float gfloat;
    gdouble *Wg64 = (gdouble *)(F.Wz + wo);
    gfloat *Wg32 = (gfloat *)(F.Wz32 + wo);
    if (MAXNZ <= 32) {
        constexpr int WIT = ((MAXNZ + 3) * MAXNZ + MZ2_THREADS - 1) / MZ2_THREADS;
        T wv[WIT];
#pragma unroll
        for (int i = 0; i < WIT; ++i) {
            const int t = threadIdx.x + i * MZ2_THREADS;
            wv[i] = t < nz * nz ? (F32 ? (T)Wg32[t] : (T)Wg64[t]) : (T)0;
        }
#pragma unroll
        for (int i = 0; i < WIT; ++i) {
            const int t = threadIdx.x + i * MZ2_THREADS;
            if (t < wn) W[t] = wv[i];
        }
    } else {
        for (int t = threadIdx.x; t < wn; t += MZ2_THREADS) W[t] = t < nz * nz ? (F32 ? (T)Wg32[t] : (T)Wg64[t]) : (T)0;
    }
    if (F32 && !std::is_same<TI, float>::value) {   // the column stays FP64 until all of the block's loads have issued
#pragma unroll
        for (int k = 0; k < MAXNZ; ++k) asm volatile("" : "+v"(vd[k]));
    }
    __syncthreads();                                   // W staged; every column of the block read
    if (!ok) return;
    T v[MAXNZ];
#pragma unroll
    for (int k = 0; k < MAXNZ; ++k) v[k] = (T)vd[k];
    // groups of four outputs (independent sums; rows past nz read zeros)
    for (int k2 = 4 * sub; k2 < nz; k2 += 4 * split) {
        T acc[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < MAXNZ; ++k)
            if (k < nz) {
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] += W[(k2 + u) * nz + k] * v[k];
            }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k2 + u < nz) out[base + (long long)(k2 + u) * nxy] = (TO)acc[u];
    }
}

// The smallest |denominator| the block met (each thread's v), into *dst by
// one atomic per block on the bit pattern (nonnegative doubles order as their
// bits), skipped unless the block lowers the stored value (which only falls).
// Every thread of the block calls it; one barrier (a wave minimum by
// shuffles, then one LDS slot per wave).
__device__ __forceinline__ void block_min_store(double v, double *dst) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    __shared__ double wmin[16];
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmin[0];
        for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = fmin(m, wmin[w]);
        if (m < __builtin_nontemporal_load(dst))
            atomicMin((unsigned long long *)dst, (unsigned long long)__double_as_longlong(m));
    }
}

// ---------------------------------------------------------------------------
// Preconditioner, per (request, alpha, M', k) slice T (nx x ny):
//   T <- Wbar_x T Wbar_y^T;  solve (Lambda_x (x) I + I (x) Lambda_y - E) T' = T;
//   T <- W_x T' W_y^T.
__device__ void block_divide(double *T, int ld, int nx, int ny, const double *lx, const double *lxi,
                             const signed char *tx, const double *ly, const double *lyi, const signed char *ty,
                             double E, double *min_den) {
    double mind = 1e300;
    for (int oo = threadIdx.x; oo < nx * ny; oo += blockDim.x) {
        const int i = oo / ny, j = oo % ny;
        const int o = i * ld + j;
        const int ti = tx[i], tj = ty[j];
        if (ti == 2 || tj == 2) continue;        // handled by the anchor of its block
        const double d = lx[i] + ly[j] - E;
        if (ti == 0 && tj == 0) {
            T[o] /= d;
            mind = fmin(mind, fabs(d));
        } else if (ti == 1 && tj == 0) {
            const double b = lxi[i], r0 = T[o], r1 = T[o + ld], det = d * d + b * b;
            T[o] = (d * r0 - b * r1) / det;
            T[o + ld] = (b * r0 + d * r1) / det;
            mind = fmin(mind, sqrt(det));
        } else if (ti == 0 && tj == 1) {
            const double b = lyi[j], r0 = T[o], r1 = T[o + 1], det = d * d + b * b;
            T[o] = (d * r0 - b * r1) / det;
            T[o + 1] = (b * r0 + d * r1) / det;
            mind = fmin(mind, sqrt(det));
        } else {
            // Both indices in complex pairs: the x and y 2x2 blocks act as two
            // commuting complex structures J1, J2; the 4x4 system splits on the
            // eigenspaces of J1 J2 into two complex divisions by
            // d + i (bx - by) and d + i (bx + by).
            const double bx = lxi[i], by = lyi[j];
            const double r00 = T[o], r01 = T[o + 1], r10 = T[o + ld], r11 = T[o + ld + 1];
            const double p00 = 0.5 * (r00 + r11), p01 = 0.5 * (r01 - r10);   // (1 + J1 J2) R / 2
            const double m00 = 0.5 * (r00 - r11), m01 = 0.5 * (r01 + r10);   // (1 - J1 J2) R / 2
            const double bp = bx - by, bm = bx + by;
            const double Dp = d * d + bp * bp, Dm = d * d + bm * bm;
            // rows of P+R: (p00, p01), (-p01, p00); of P-R: (m00, m01), (m01, -m00)
            T[o] = (d * p00 + bp * p01) / Dp + (d * m00 - bm * m01) / Dm;
            T[o + 1] = (d * p01 - bp * p00) / Dp + (d * m01 + bm * m00) / Dm;
            T[o + ld] = (-d * p01 + bp * p00) / Dp + (d * m01 + bm * m00) / Dm;
            T[o + ld + 1] = (d * p00 + bp * p01) / Dp + (-d * m00 + bm * m01) / Dm;
            mind = fmin(mind, sqrt(fmin(Dp, Dm)));
        }
    }
    if (min_den) block_min_store(mind, min_den);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Preconditioner x-y slice on FP64 MFMA (v_mfma_f64_16x16x4f64).  The slice is
// held in LDS zero-padded to multiples of 16 (row stride ld); each of the 4
// waves accumulates its 16x16 output tiles in registers over the whole K
// range, then, after a barrier, writes them back in place.
// Operand layout of the 16x16x4 FP64 MFMA: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[l/16 + 4v][l%16], v = 0..3 (each 64-bit
// accumulator register holds four rows that are 4 apart; the FP32 16x16
// MFMAs instead hold rows 4(l/16) + v).
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int XYM_MAXT = 16;        // tiles per wave: (128/16)^2 / 4

// T <- Wm T (LEFT, Wm: nx x nx) or T <- T Wm^T (!LEFT, Wm: ny x ny); at most
// MAXT output tiles per wave.
template <bool LEFT, int MAXT, int NW>
__device__ void mfma_slice_mult(double *T, int ld, int nxp, int nyp, const double *__restrict__ Wm, int nw) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int tcols = nyp >> 4, ntiles = (nxp >> 4) * tcols;
    const int K = LEFT ? nxp : nyp;
    dbl4 acc[MAXT];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int kk = k0 + k4;
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int t = wave + NW * q;
            if (t < ntiles) {
                const int i0 = (t / tcols) << 4, j0 = (t % tcols) << 4;
                double a, b;
                if (LEFT) {
                    const int row = i0 + r16;
                    a = (row < nw && kk < nw) ? Wm[(size_t)row * nw + kk] : 0.0;
                    b = T[kk * ld + j0 + r16];
                } else {
                    const int col = j0 + r16;
                    a = T[(i0 + r16) * ld + kk];
                    b = (col < nw && kk < nw) ? Wm[(size_t)col * nw + kk] : 0.0;
                }
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int t = wave + NW * q;
        if (t < ntiles) {
            const int i0 = (t / tcols) << 4, j0 = (t % tcols) << 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) T[(i0 + k4 + 4 * v) * ld + j0 + r16] = acc[q][v];
        }
    }
    __syncthreads();
}

template <int MAXT, int NW>
__global__ void __launch_bounds__(NW * 64) k_xy_mfma(const ProblemDev *__restrict__ pd,
                                                        const PrecDev *__restrict__ pr,
                                                        const double *__restrict__ Evec,
                                                        const int *__restrict__ active, double *data,
                                                        double *min_den) {
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    const int a = blockIdx.y / MAXM, iM = blockIdx.y % MAXM;
    if (iM >= pd->nM) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int k = blockIdx.x;
    const int nz = C.z.n, nx = C.x.n, ny = C.y.n;
    if (k >= nz) return;
    const int nxp = (nx + 15) & ~15, nyp = (ny + 15) & ~15, ld = nyp + 4;
    extern __shared__ double T[];
    double *g = data + (long long)req * pd->N + C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    for (int t = threadIdx.x; t < nxp * ld; t += NW * 64) {
        const int i = t / ld, j = t % ld;
        T[t] = (i < nx && j < ny) ? g[i * ny + j] : 0.0;
    }
    __syncthreads();
    const size_t fx = (size_t)iM * nz + k;
    const double *Wbx = F.Wx + fx * 2 * nx * nx, *Wx = Wbx + (size_t)nx * nx;
    const double *Wby = F.Wy + fx * 2 * ny * ny, *Wy = Wby + (size_t)ny * ny;
    mfma_slice_mult<true, MAXT, NW>(T, ld, nxp, nyp, Wbx, nx);
    mfma_slice_mult<false, MAXT, NW>(T, ld, nxp, nyp, Wby, ny);
    block_divide(T, ld, nx, ny, F.lx + fx * nx, F.lxi + fx * nx, F.tx + fx * nx, F.ly + fx * ny, F.lyi + fx * ny,
                 F.ty + fx * ny, Evec[req], min_den ? min_den + req : nullptr);
    mfma_slice_mult<true, MAXT, NW>(T, ld, nxp, nyp, Wx, nx);
    mfma_slice_mult<false, MAXT, NW>(T, ld, nxp, nyp, Wy, ny);
    for (int t = threadIdx.x; t < nx * ny; t += NW * 64) g[t] = T[(t / ny) * ld + t % ny];
}

// ---------------------------------------------------------------------------
// Staged x-y products, for slices wider than one block's LDS tile of the
// fused kernel holds: each of the four products is a batched FP64 MFMA GEMM over
// all (request, alpha, M', k) slices with 32 x 32 output tiles (a 16 x 16 tile
// per wave), reading one buffer and writing the other; the divide is a pass of
// its own in between.  Slices are numbered alpha-major, then M', then k.
constexpr int SG_T = 32, SG_KC = 32;

// Tiles of a slice side n at tile width bt: with 32 x 32 tiles a side of
// 32 m + 1 (the quintic bases of 3K + 1 functions with K a multiple of 32: 97,
// 193) takes m tiles, the last of which also computes the leftover row or
// column with vector FMAs, instead of an (m+1)-th tile holding one useful line.
__host__ __device__ inline int sg_tiles(int n, int bt) {
    return bt == 32 && n > bt && n % bt == 1 ? n / bt : (n + bt - 1) / bt;
}

__device__ __forceinline__ bool slice_decode(const ProblemDev *pd, int s, int &a, int &iM, int &k) {
    a = 0;
    while (a < 3 && s >= pd->nM * pd->comp[a].z.n) {
        s -= pd->nM * pd->comp[a].z.n;
        ++a;
    }
    if (a >= 3) return false;
    iM = s / pd->comp[a].z.n;
    k = s % pd->comp[a].z.n;
    return true;
}

// 1/d in FP64: the hardware reciprocal estimate refined by two Newton steps
// r <- r + r (1 - d r), each doubling the correct bits (within an ulp or two of
// the rounded quotient, at a fraction of an IEEE division's cost).
__device__ __forceinline__ double rcp_newton(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

// One element of the divided slice, (Lambda_x (x) I + I (x) Lambda_y - E)^-1 T
// at (i, j), from T and the 2x2 / 4x4 blocks of complex pairs it belongs to
// (the same closed forms as block_divide); mind tracks min |denominator|.
template <class TT>
__device__ __forceinline__ double divided_at(const TT *__restrict__ T, int ld, int i, int j,
                                             const double *__restrict__ lx, const double *__restrict__ lxi,
                                             const signed char *__restrict__ tx, const double *__restrict__ ly,
                                             const double *__restrict__ lyi, const signed char *__restrict__ ty,
                                             double E, double &mind) {
    const int ti = tx[i], tj = ty[j];
    const int i0 = ti == 2 ? i - 1 : i, j0 = tj == 2 ? j - 1 : j;
    const double d = lx[i0] + ly[j0] - E;
    if (ti == 0 && tj == 0) {
        mind = fmin(mind, fabs(d));
        return (double)T[(size_t)i * ld + j] / d;
    }
    if (tj == 0) {
        const double b = lxi[i0], r0 = T[(size_t)i0 * ld + j], r1 = T[(size_t)(i0 + 1) * ld + j], det = d * d + b * b;
        mind = fmin(mind, sqrt(det));
        return ti == 1 ? (d * r0 - b * r1) / det : (b * r0 + d * r1) / det;
    }
    if (ti == 0) {
        const double b = lyi[j0], r0 = T[(size_t)i * ld + j0], r1 = T[(size_t)i * ld + j0 + 1], det = d * d + b * b;
        mind = fmin(mind, sqrt(det));
        return tj == 1 ? (d * r0 - b * r1) / det : (b * r0 + d * r1) / det;
    }
    const double bx = lxi[i0], by = lyi[j0];
    const double r00 = T[(size_t)i0 * ld + j0], r01 = T[(size_t)i0 * ld + j0 + 1];
    const double r10 = T[(size_t)(i0 + 1) * ld + j0], r11 = T[(size_t)(i0 + 1) * ld + j0 + 1];
    const double p00 = 0.5 * (r00 + r11), p01 = 0.5 * (r01 - r10);
    const double m00 = 0.5 * (r00 - r11), m01 = 0.5 * (r01 + r10);
    const double bp = bx - by, bm = bx + by;
    const double Dp = d * d + bp * bp, Dm = d * d + bm * bm;
    mind = fmin(mind, sqrt(fmin(Dp, Dm)));
    if (ti == 1 && tj == 1) return (d * p00 + bp * p01) / Dp + (d * m00 - bm * m01) / Dm;
    if (ti == 1) return (d * p01 - bp * p00) / Dp + (d * m01 + bm * m00) / Dm;
    if (tj == 1) return (-d * p01 + bp * p00) / Dp + (d * m01 + bm * m00) / Dm;
    return (d * p00 + bp * p01) / Dp + (-d * m00 + bm * m01) / Dm;
}

// LEFT: out = W in (W: nx x nx); RIGHT: out = in W^T (W: ny x ny); which
// selects Wbar (0) or W (1) of the slice's pencil.  DIV (LEFT only): the
// input is divided by lambda_x + lambda_y - E element by element as it is
// loaded (the divide of the tensor trick between the two product pairs);
// min_den (may be null) receives the smallest |denominator| met.  Grid:
// (slices, tiles, requests); 256 threads.  Slices run fastest because the
// hardware deals consecutive blocks to the 8 XCDs in turn: with a slice count
// that is a multiple of 8, every tile of a slice (and every request's copy of
// it) lands on one XCD and shares that XCD's L2 for the slice's W and data.
// JZ (LEFT only, coupled preconditioner): the "slice" is a whole component,
// the n_M n_z x n_x n_y matrix of its [M'][z] rows, and W its joint z matrix
// (grid.y = 3); in and out must not overlap.
// DIVOUT (right products only): each output element whose x and y
// eigenvalues are both real is divided by lambda_x + lambda_y - E as it is
// stored (the elements of complex pairs are stored undivided for
// k_divide_pairs), so the next left product needs no divide.
template <bool LEFT, bool DIV, bool JZ = false, int BT = SG_T, bool DIVOUT = false>
__global__ void __launch_bounds__(256) k_slice_gemm(const ProblemDev *__restrict__ pd, const PrecDev *__restrict__ pr,
                                                    const double *__restrict__ Evec,
                                                    const int *__restrict__ active, int which,
                                                    const double *__restrict__ in, double *__restrict__ out,
                                                    double *min_den) {
    static_assert(!JZ || (LEFT && !DIV), "joint z products are plain left products");
    static_assert(!DIVOUT || (!LEFT && !DIV && !JZ), "the divide on store follows a right product");
    static_assert(BT == 32 || BT == 64, "block tile 32 x 32 (one 16 x 16 MFMA tile per wave) or 64 x 64 (2 x 2)");
    constexpr int WT = BT / 32;               // MFMA tiles per wave in each direction
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    int a, iM, k;
    if (JZ) {
        a = blockIdx.y;
        iM = k = 0;
    } else if (!slice_decode(pd, blockIdx.x, a, iM, k)) {
        return;
    }
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nz = C.z.n;
    const int nx = JZ ? pd->nM * nz : C.x.n, ny = JZ ? C.nxy : C.y.n;
    const int tr = JZ ? (nx + BT - 1) / BT : sg_tiles(nx, BT), tc = JZ ? (ny + BT - 1) / BT : sg_tiles(ny, BT);
    const int t = JZ ? blockIdx.x : blockIdx.y;
    if (t >= tr * tc) return;
    const int i0 = (t / tc) * BT, j0 = (t % tc) * BT;
    // the last tile of a side bt m + 1 also computes line n - 1 (see sg_tiles)
    constexpr bool EXT = !JZ && BT == 32;
    const bool erow = EXT && i0 + BT == nx - 1 && nx % BT == 1, ecol = EXT && j0 + BT == ny - 1 && ny % BT == 1;
    const size_t fx = (size_t)iM * nz + k;
    const double *Wm = JZ     ? F.Zj + (size_t)which * nx * nx
                       : LEFT ? F.Wx + (fx * 2 + which) * nx * nx
                              : F.Wy + (fx * 2 + which) * ny * ny;
    const long long off = (long long)req * pd->N + C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    const double *g = in + off;
    double *o = out + off;
    const int K = LEFT ? nx : ny;
    const double E = DIV ? Evec[req] : 0.0;
    const double E2 = DIVOUT ? Evec[req] : 0.0;
    double mind = 1e300;
    // the operand tiles, one buffer
    __shared__ double sg_buf[BT * (SG_KC + 1) + SG_KC * (BT + 1)];
    double (*As)[SG_KC + 1] = reinterpret_cast<double (*)[SG_KC + 1]>(sg_buf);              // [row][k]
    double (*Bs)[BT + 1] = reinterpret_cast<double (*)[BT + 1]>(sg_buf + BT * (SG_KC + 1));   // [k][col]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, k4 = lane >> 4, wi = wave >> 1, wj = wave & 1;
    constexpr int PER = BT * SG_KC / 256;   // A and B values per thread per chunk
    double ra[PER], rb[PER];
    // leftover line: A's row nx - 1 (threads 0..KC-1) and B's column ny - 1
    // (threads 64..64+KC-1) of the chunk; threads 0..BT-1 sum row outputs,
    // BT..2BT-1 column outputs, 2BT the corner
    __shared__ double Ae[SG_KC], Be[SG_KC];
    double rae = 0.0, rbe = 0.0, ext = 0.0;
    // the next chunk is fetched into registers while the current one is multiplied
    // DIV: the x eigenvalue data of all K rows staged in LDS once, and the y data
    // of this thread's column (a thread's B elements share one column: 256 is a
    // multiple of BT) in registers; the divide of a real (lambda_x, lambda_y) pair
    // then reads nothing but its element, complex pairs take divided_at
    constexpr int DIV_ROWS = 256;
    __shared__ double sLx[DIV ? DIV_ROWS : 1];
    __shared__ signed char sTx[DIV ? DIV_ROWS : 1];
    const bool staged = DIV && K <= DIV_ROWS;
    double ly_c = 0.0;
    int ty_c = 1;
    if (DIV) {
        // (K <= 256 when staged: one row per thread) through global-memory
        // pointers, every load before the LDS writes: a flat load may alias LDS
        // and would wait before each write
        typedef const __attribute__((address_space(1))) double gdouble;
        typedef const __attribute__((address_space(1))) signed char gschar;
        const int r = threadIdx.x;
        const bool st = staged && r < K;
        const double lxv = st ? ((gdouble *)F.lx)[fx * nx + r] : 0.0;
        const signed char txv = st ? ((gschar *)F.tx)[fx * nx + r] : (signed char)0;
        const int jc = j0 + (int)threadIdx.x % BT;
        if (jc < ny) {
            ly_c = ((gdouble *)F.ly)[fx * ny + jc];
            ty_c = ((gschar *)F.ty)[fx * ny + jc];
        }
        if (st) {
            sLx[r] = lxv;
            sTx[r] = txv;
        }
        __syncthreads();
    }
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int r = e / SG_KC, c = e % SG_KC;          // A[r][c]: row i0 + r, k0 + c
            const int row = i0 + r, kk = k0 + c;
            double av = 0.0;
            if (row < nx && kk < K) av = LEFT ? Wm[(size_t)row * nx + kk] : g[(size_t)row * ny + kk];
            ra[q] = av;
            double bv = 0.0;
            if (LEFT) {
                const int kb = e / BT, cb = e % BT;          // B[kb][cb] = in[k0 + kb][j0 + cb]
                // raw values only: the divide (DIV) is applied when the chunk is
                // stashed, so that all loads of a chunk are in flight together
                if (k0 + kb < K && j0 + cb < ny) bv = g[(size_t)(k0 + kb) * ny + j0 + cb];
            } else {
                const int cb = e / SG_KC, kb = e % SG_KC;    // B[kb][cb] = W[j0 + cb][k0 + kb]
                if (k0 + kb < K && j0 + cb < ny) bv = Wm[(size_t)(j0 + cb) * ny + k0 + kb];
            }
            rb[q] = bv;
        }
        if (erow && threadIdx.x < SG_KC) {
            const int kk = k0 + threadIdx.x;
            rae = kk < K ? (LEFT ? Wm[(size_t)(nx - 1) * nx + kk] : g[(size_t)(nx - 1) * ny + kk]) : 0.0;
        }
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC) {
            const int kb = k0 + (int)threadIdx.x - 64;
            rbe = kb < K ? (LEFT ? g[(size_t)kb * ny + ny - 1] : Wm[(size_t)(ny - 1) * ny + kb]) : 0.0;
        }
    };
    // DIV: divide the fetched chunk in registers (after the products of the
    // previous chunk, so its loads have landed)
    auto divide = [&](int k0) {
        if (!DIV) return;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int kb = e / BT, cb = e % BT;
            if (k0 + kb < K && j0 + cb < ny) {
                if (staged && ty_c == 0 && sTx[k0 + kb] == 0) {
                    const double d = sLx[k0 + kb] + ly_c - E;
                    mind = fmin(mind, fabs(d));
                    rb[q] = rb[q] * rcp_newton(d);
                } else {                           // complex pairs: closed forms over their 2x2 / 4x4 blocks
                    rb[q] = divided_at(g, ny, k0 + kb, j0 + cb, F.lx + fx * nx, F.lxi + fx * nx, F.tx + fx * nx,
                                       F.ly + fx * ny, F.lyi + fx * ny, F.ty + fx * ny, E, mind);
                }
            }
        }
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC && k0 + (int)threadIdx.x - 64 < K)
            rbe = divided_at(g, ny, k0 + (int)threadIdx.x - 64, ny - 1, F.lx + fx * nx, F.lxi + fx * nx,
                             F.tx + fx * nx, F.ly + fx * ny, F.lyi + fx * ny, F.ty + fx * ny, E, mind);
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            As[e / SG_KC][e % SG_KC] = ra[q];
            if (LEFT) Bs[e / BT][e % BT] = rb[q];
            else Bs[e % SG_KC][e / SG_KC] = rb[q];
        }
        if (erow && threadIdx.x < SG_KC) Ae[threadIdx.x] = rae;
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC) Be[threadIdx.x - 64] = rbe;
    };
    // DIVOUT: the eigenvalues and types of the tile's rows and columns,
    // requested now so that they arrive during the products (a type of 1 marks
    // a line outside the slice, which is not divided); through LDS, written
    // here and read after the products (the first barrier of the chunk loop
    // orders them), so that no register is held over the products
    __shared__ double dv_sl[DIVOUT ? BT : 1], dv_cl[DIVOUT ? BT : 1];
    __shared__ int dv_st[DIVOUT ? BT : 1], dv_ct[DIVOUT ? BT : 1];
    if (DIVOUT && threadIdx.x < BT) {
        const int row = i0 + (int)threadIdx.x;
        dv_sl[threadIdx.x] = row < nx ? F.lx[fx * nx + row] : 0.0;
        dv_st[threadIdx.x] = row < nx ? F.tx[fx * nx + row] : 1;
    } else if (DIVOUT && threadIdx.x < 2 * BT) {
        const int c = (int)threadIdx.x - BT, col = j0 + c;
        dv_cl[c] = col < ny ? F.ly[fx * ny + col] : 0.0;
        dv_ct[c] = col < ny ? F.ty[fx * ny + col] : 1;
    }
    // wave (wi, wj) owns the (16 WT) x (16 WT) block at rows 16 WT wi, columns 16 WT wj
    dbl4 acc[WT][WT];
#pragma unroll
    for (int ti = 0; ti < WT; ++ti)
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) acc[ti][tj] = dbl4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    divide(0);
    for (int k0 = 0; k0 < K; k0 += SG_KC) {
        stash();
        __syncthreads();
        if (k0 + SG_KC < K) fetch(k0 + SG_KC);
#pragma unroll
        for (int kk = 0; kk < SG_KC; kk += 4) {
            if (kk >= K - k0) break;            // the zero padding past K
            double av[WT], bv[WT];
#pragma unroll
            for (int ti = 0; ti < WT; ++ti) av[ti] = As[16 * (WT * wi + ti) + r16][kk + k4];
#pragma unroll
            for (int tj = 0; tj < WT; ++tj) bv[tj] = Bs[kk + k4][16 * (WT * wj + tj) + r16];
#pragma unroll
            for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                for (int tj = 0; tj < WT; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
        }
        if (erow || ecol) {
            const int tx = threadIdx.x, kn = min(SG_KC, K - k0);
            if (erow && tx < BT)
                for (int kk = 0; kk < kn; ++kk) ext += Ae[kk] * Bs[kk][tx];
            else if (ecol && tx >= BT && tx < 2 * BT)
                for (int kk = 0; kk < kn; ++kk) ext += As[tx - BT][kk] * Be[kk];
            else if (erow && ecol && tx == 2 * BT)
                for (int kk = 0; kk < kn; ++kk) ext += Ae[kk] * Be[kk];
        }
        if (k0 + SG_KC < K) divide(k0 + SG_KC);
        __syncthreads();
    }
    // DIVOUT: the divisor of an element (i, j), real eigenvalue pairs only
    // (the lane's rows and columns were read before the products)
    auto divout = [&](int row, int col, double v) {
        if (!DIVOUT) return v;
        const int ti = F.tx[fx * nx + row], tj = F.ty[fx * ny + col];
        if (ti != 0 || tj != 0) return v;                  // complex pairs: k_divide_pairs
        const double d = F.lx[fx * nx + row] + F.ly[fx * ny + col] - E2;
        mind = fmin(mind, fabs(d));
        return v * rcp_newton(d);
    };
    {
        // stores straight from the accumulators; DIVOUT divides on the way, with
        // the rows' and the lane's columns' eigenvalues from LDS
        double cl[WT];
        int ct[WT];
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) {
            cl[tj] = DIVOUT ? dv_cl[16 * (WT * wj + tj) + r16] : 0.0;
            ct[tj] = DIVOUT ? dv_ct[16 * (WT * wj + tj) + r16] : 1;
        }
#pragma unroll
        for (int ti = 0; ti < WT; ++ti)
#pragma unroll
            for (int tj = 0; tj < WT; ++tj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rl = 16 * (WT * wi + ti) + k4 + 4 * v;
                    const int row = i0 + rl, col = j0 + 16 * (WT * wj + tj) + r16;
                    if (row < nx && col < ny) {
                        double val = acc[ti][tj][v];
                        if (DIVOUT && (dv_st[rl] | ct[tj]) == 0) {
                            const double d = dv_sl[rl] + cl[tj] - E2;
                            mind = fmin(mind, fabs(d));
                            val *= rcp_newton(d);
                        }
                        o[(size_t)row * ny + col] = val;
                    }
                }
    }
    if (erow || ecol) {
        const int tx = threadIdx.x;
        if (erow && tx < BT && j0 + tx < ny) o[(size_t)(nx - 1) * ny + j0 + tx] = divout(nx - 1, j0 + tx, ext);
        else if (ecol && tx >= BT && tx < 2 * BT && i0 + tx - BT < nx)
            o[(size_t)(i0 + tx - BT) * ny + ny - 1] = divout(i0 + tx - BT, ny - 1, ext);
        else if (erow && ecol && tx == 2 * BT) o[(size_t)(nx - 1) * ny + ny - 1] = divout(nx - 1, ny - 1, ext);
    }
    if ((DIV || DIVOUT) && min_den) block_min_store(mind, min_den + req);
}


// The divide of the elements in complex-conjugate eigenpair blocks, in place,
// after a right product stored with DIVOUT (which divided every element of
// two real eigenvalues): the 2 x 2 blocks of an x pair (rows i, i + 1) or a
// y pair (columns j, j + 1) and the 4 x 4 blocks of both, by the closed forms
// of block_divide.  One block per (slice with complex pairs, request).
constexpr int DP_MAXP = 512;

template <class TD>
__global__ void __launch_bounds__(256) k_divide_pairs(const ProblemDev *__restrict__ pd, const PrecDev *__restrict__ pr,
                                                      const double *__restrict__ Evec, const int *__restrict__ active,
                                                      TD *data, double *min_den) {
    const int req = blockIdx.y;
    if (active && !active[req]) return;
    int a, iM, k;
    if (!slice_decode(pd, pr->pair_slices[blockIdx.x], a, iM, k)) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nx = C.x.n, ny = C.y.n, nz = C.z.n;
    const size_t fx = (size_t)iM * nz + k;
    const double *lx = F.lx + fx * nx, *lxi = F.lxi + fx * nx, *ly = F.ly + fx * ny, *lyi = F.lyi + fx * ny;
    const signed char *tx = F.tx + fx * nx, *ty = F.ty + fx * ny;
    __shared__ int xs[DP_MAXP], ys[DP_MAXP];
    __shared__ int nxp, nyp;
    if (threadIdx.x == 0) nxp = nyp = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < nx; i += 256)
        if (tx[i] == 1) {
            const int s = atomicAdd(&nxp, 1);
            if (s < DP_MAXP) xs[s] = i;
        }
    for (int j = threadIdx.x; j < ny; j += 256)
        if (ty[j] == 1) {
            const int s = atomicAdd(&nyp, 1);
            if (s < DP_MAXP) ys[s] = j;
        }
    __syncthreads();
    const int px = min(nxp, DP_MAXP), py = min(nyp, DP_MAXP);
    if (px == 0 && py == 0) return;
    TD *T = data + (long long)req * pd->N + C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    const double E = Evec[req];
    double mind = 1e300;
    // x pairs: rows i, i + 1 against every column (4 x 4 where the column is in a pair too)
    for (int t = threadIdx.x; t < px * ny; t += 256) {
        const int i = xs[t / ny], j = t % ny;
        const int tj = ty[j];
        if (tj == 2) continue;
        const double d = lx[i] + ly[j] - E;
        const int o = i * ny + j;
        if (tj == 0) {
            const double b = lxi[i], r0 = T[o], r1 = T[o + ny], det = d * d + b * b;
            T[o] = (TD)((d * r0 - b * r1) / det);
            T[o + ny] = (TD)((b * r0 + d * r1) / det);
            mind = fmin(mind, sqrt(det));
        } else {
            const double bx = lxi[i], by = lyi[j];
            const double r00 = T[o], r01 = T[o + 1], r10 = T[o + ny], r11 = T[o + ny + 1];
            const double p00 = 0.5 * (r00 + r11), p01 = 0.5 * (r01 - r10);
            const double m00 = 0.5 * (r00 - r11), m01 = 0.5 * (r01 + r10);
            const double bp = bx - by, bm = bx + by;
            const double Dp = d * d + bp * bp, Dm = d * d + bm * bm;
            T[o] = (TD)((d * p00 + bp * p01) / Dp + (d * m00 - bm * m01) / Dm);
            T[o + 1] = (TD)((d * p01 - bp * p00) / Dp + (d * m01 + bm * m00) / Dm);
            T[o + ny] = (TD)((-d * p01 + bp * p00) / Dp + (d * m01 + bm * m00) / Dm);
            T[o + ny + 1] = (TD)((d * p00 + bp * p01) / Dp + (-d * m00 + bm * m01) / Dm);
            mind = fmin(mind, sqrt(fmin(Dp, Dm)));
        }
    }
    // y pairs: columns j, j + 1 in the rows of real x eigenvalues
    for (int t = threadIdx.x; t < nx * py; t += 256) {
        const int i = t / py, j = ys[t % py];
        if (tx[i] != 0) continue;
        const double d = lx[i] + ly[j] - E;
        const int o = i * ny + j;
        const double b = lyi[j], r0 = T[o], r1 = T[o + 1], det = d * d + b * b;
        T[o] = (TD)((d * r0 - b * r1) / det);
        T[o + 1] = (TD)((b * r0 + d * r1) / det);
        mind = fmin(mind, sqrt(det));
    }
    if (min_den) block_min_store(mind, min_den + req);
}

// ---------------------------------------------------------------------------
// Reduced-precision preconditioner products (the divide stays FP64).
//   MODE 1: FP32 MFMA v_mfma_f32_16x16x4f32 (lane layout as the FP64 one).
//   MODE 2: BF16x3: each operand a = a_hi + a_mid (+ a_lo) in bfloat16, the
//           product taken as a_hi b_hi + a_hi b_mid + a_mid b_hi with FP32
//           accumulation (Henry, Tang, Heinecke, ARITH 2019), on
//           v_mfma_f32_16x16x16bf16_1k: lane l supplies A[l%16][4(l/16)+0..3]
//           and B[4(l/16)+0..3][l%16]; D as above.
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short sht4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f32_to_bf16(float f) {   // round to nearest even
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ __forceinline__ void split_bf16(float a, short &hi, short &mid) {
    const unsigned short h = f32_to_bf16(a);
    hi = (short)h;
    mid = (short)f32_to_bf16(a - bf16_to_f32(h));
}

template <bool LEFT, int MAXT, int NW>
__device__ void mfma32_slice_mult(float *T, int ld, int nxp, int nyp, const float *__restrict__ Wm, int nw) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int tcols = nyp >> 4, ntiles = (nxp >> 4) * tcols;
    const int K = LEFT ? nxp : nyp;
    flt4 acc[MAXT];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) acc[q] = flt4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int kk = k0 + k4;
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int t = wave + NW * q;
            if (t < ntiles) {
                const int i0 = (t / tcols) << 4, j0 = (t % tcols) << 4;
                float a, b;
                if (LEFT) {
                    const int row = i0 + r16;
                    a = (row < nw && kk < nw) ? Wm[(size_t)row * nw + kk] : 0.f;
                    b = T[kk * ld + j0 + r16];
                } else {
                    const int col = j0 + r16;
                    a = T[(i0 + r16) * ld + kk];
                    b = (col < nw && kk < nw) ? Wm[(size_t)col * nw + kk] : 0.f;
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int t = wave + NW * q;
        if (t < ntiles) {
            const int i0 = (t / tcols) << 4, j0 = (t % tcols) << 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) T[(i0 + 4 * k4 + v) * ld + j0 + r16] = acc[q][v];
        }
    }
    __syncthreads();
}

// W16: bfloat16 planes of Wm, [0] = hi, [1] = mid (plane stride pstride).
template <bool LEFT, int MAXT, int NW>
__device__ void mfma_bf3_slice_mult(float *T, int ld, int nxp, int nyp, const unsigned short *__restrict__ W16,
                                    size_t pstride, int nw) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4;
    const int tcols = nyp >> 4, ntiles = (nxp >> 4) * tcols;
    const int K = LEFT ? nxp : nyp;
    flt4 acc[MAXT];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) acc[q] = flt4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int kk = k0 + g4;
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int t = wave + NW * q;
            if (t < ntiles) {
                const int i0 = (t / tcols) << 4, j0 = (t % tcols) << 4;
                sht4 dhi, dmid, whi, wmid;       // data and factor operands
                const int wrow = LEFT ? i0 + r16 : j0 + r16;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kc = kk + e;
                    const bool ok = wrow < nw && kc < nw;
                    whi[e] = ok ? (short)W16[(size_t)wrow * nw + kc] : (short)0;
                    wmid[e] = ok ? (short)W16[pstride + (size_t)wrow * nw + kc] : (short)0;
                    const float dv = LEFT ? T[kc * ld + j0 + r16] : T[(i0 + r16) * ld + kc];
                    short h, m;
                    split_bf16(dv, h, m);
                    dhi[e] = h;
                    dmid[e] = m;
                }
                if (LEFT) {      // A = W, B = T
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wmid, dhi, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(whi, dmid, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(whi, dhi, acc[q], 0, 0, 0);
                } else {         // A = T, B = W^T
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dmid, whi, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dhi, wmid, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dhi, whi, acc[q], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int t = wave + NW * q;
        if (t < ntiles) {
            const int i0 = (t / tcols) << 4, j0 = (t % tcols) << 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) T[(i0 + 4 * (lane >> 4) + v) * ld + j0 + r16] = acc[q][v];
        }
    }
    __syncthreads();
}

// The FP64 block divide on an FP32 slice: values are widened, divided, narrowed.
__device__ void block_divide_f32(float *T, int ld, int nx, int ny, const double *lx, const double *lxi,
                                 const signed char *tx, const double *ly, const double *lyi, const signed char *ty,
                                 double E) {
    for (int oo = threadIdx.x; oo < nx * ny; oo += blockDim.x) {
        const int i = oo / ny, j = oo % ny;
        const int o = i * ld + j;
        const int ti = tx[i], tj = ty[j];
        if (ti == 2 || tj == 2) continue;
        const double d = lx[i] + ly[j] - E;
        if (ti == 0 && tj == 0) {
            T[o] = (float)((double)T[o] / d);
        } else if (ti == 1 && tj == 0) {
            const double b = lxi[i], r0 = T[o], r1 = T[o + ld], det = d * d + b * b;
            T[o] = (float)((d * r0 - b * r1) / det);
            T[o + ld] = (float)((b * r0 + d * r1) / det);
        } else if (ti == 0 && tj == 1) {
            const double b = lyi[j], r0 = T[o], r1 = T[o + 1], det = d * d + b * b;
            T[o] = (float)((d * r0 - b * r1) / det);
            T[o + 1] = (float)((b * r0 + d * r1) / det);
        } else {
            const double bx = lxi[i], by = lyi[j];
            const double r00 = T[o], r01 = T[o + 1], r10 = T[o + ld], r11 = T[o + ld + 1];
            const double p00 = 0.5 * (r00 + r11), p01 = 0.5 * (r01 - r10);
            const double m00 = 0.5 * (r00 - r11), m01 = 0.5 * (r01 + r10);
            const double bp = bx - by, bm = bx + by;
            const double Dp = d * d + bp * bp, Dm = d * d + bm * bm;
            T[o] = (float)((d * p00 + bp * p01) / Dp + (d * m00 - bm * m01) / Dm);
            T[o + 1] = (float)((d * p01 - bp * p00) / Dp + (d * m01 + bm * m00) / Dm);
            T[o + ld] = (float)((-d * p01 + bp * p00) / Dp + (d * m01 + bm * m00) / Dm);
            T[o + ld + 1] = (float)((d * p00 + bp * p01) / Dp + (-d * m00 + bm * m01) / Dm);
        }
    }
    __syncthreads();
}

// Staged x-y products in reduced precision with FP32 storage between them:
// the tiling of k_slice_gemm (BT x BT block tiles, WT x WT 16 x 16 MFMA tiles
// per wave, K in chunks of SG_KC with the next chunk fetched during the
// products) on FP32 MFMA (MODE 1: v_mfma_f32_16x16x4f32) or BF16x3 MFMA
// (MODE 2: operands split into bfloat16 hi + mid as they are read, three
// products, FP32 sums).  TI / TO: element types of in and out (FP32 between
// the products; FP64 at the ends of the coupled variant).  DIVOUT (right
// products only): each output element whose x and y eigenvalues are both real
// is divided in FP64 by lambda_x + lambda_y - E as it is stored, then rounded
// to FP32 (the elements of complex pairs are stored undivided for
// k_divide_pairs), so the next left product needs no divide.
template <bool LEFT, int MODE, int BT, class TI, class TO, bool DIVOUT = false>
__global__ void __launch_bounds__(256) k_slice_gemm_f32(const ProblemDev *__restrict__ pd,
                                                        const PrecDev *__restrict__ pr,
                                                        const double *__restrict__ Evec,
                                                        const int *__restrict__ active, int which,
                                                        const TI *__restrict__ in, TO *__restrict__ out) {
    static_assert(BT == 32 || BT == 64, "block tile 32 x 32 or 64 x 64");
    static_assert(!DIVOUT || !LEFT, "the divide on store follows a right product");
    constexpr int WT = BT / 32;
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    int a, iM, k;
    if (!slice_decode(pd, blockIdx.x, a, iM, k)) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nz = C.z.n, nx = C.x.n, ny = C.y.n;
    const int tr = sg_tiles(nx, BT), tc = sg_tiles(ny, BT);
    const int t = blockIdx.y;
    if (t >= tr * tc) return;
    const int i0 = (t / tc) * BT, j0 = (t % tc) * BT;
    constexpr bool EXT = BT == 32;
    const bool erow = EXT && i0 + BT == nx - 1 && nx % BT == 1, ecol = EXT && j0 + BT == ny - 1 && ny % BT == 1;
    const size_t fx = (size_t)iM * nz + k;
    const float *Wm = LEFT ? F.Wx32 + (fx * 2 + which) * nx * nx : F.Wy32 + (fx * 2 + which) * ny * ny;
    const long long off = (long long)req * pd->N + C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    const TI *g = in + off;
    TO *o = out + off;
    const int K = LEFT ? nx : ny;
    const double E = DIVOUT ? Evec[req] : 0.0;
    // the operand tiles, one buffer: DIVOUT reuses it for the output tile
    __shared__ float sg32[BT * (SG_KC + 1) + SG_KC * (BT + 1)];
    static_assert(BT * (SG_KC + 1) + SG_KC * (BT + 1) >= BT * (BT + 1), "output tile fits the operand tiles");
    float (*As)[SG_KC + 1] = reinterpret_cast<float (*)[SG_KC + 1]>(sg32);              // [row][k]
    float (*Bs)[BT + 1] = reinterpret_cast<float (*)[BT + 1]>(sg32 + BT * (SG_KC + 1));   // [k][col]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, k4 = lane >> 4, wi = wave >> 1, wj = wave & 1;
    constexpr int PER = BT * SG_KC / 256;
    float ra[PER], rb[PER];
    __shared__ float Ae[SG_KC], Be[SG_KC];
    float rae = 0.f, ext = 0.f, rbe = 0.f;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int r = e / SG_KC, c = e % SG_KC;
            const int row = i0 + r, kk = k0 + c;
            float av = 0.f;
            if (row < nx && kk < K) av = LEFT ? Wm[(size_t)row * nx + kk] : (float)g[(size_t)row * ny + kk];
            ra[q] = av;
            float bv = 0.f;
            if (LEFT) {
                const int kb = e / BT, cb = e % BT;
                if (k0 + kb < K && j0 + cb < ny) bv = (float)g[(size_t)(k0 + kb) * ny + j0 + cb];
            } else {
                const int cb = e / SG_KC, kb = e % SG_KC;
                if (k0 + kb < K && j0 + cb < ny) bv = Wm[(size_t)(j0 + cb) * ny + k0 + kb];
            }
            rb[q] = bv;
        }
        if (erow && threadIdx.x < SG_KC) {
            const int kk = k0 + threadIdx.x;
            rae = kk < K ? (LEFT ? Wm[(size_t)(nx - 1) * nx + kk] : (float)g[(size_t)(nx - 1) * ny + kk]) : 0.f;
        }
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC) {
            const int kb = k0 + (int)threadIdx.x - 64;
            rbe = kb < K ? (LEFT ? (float)g[(size_t)kb * ny + ny - 1] : Wm[(size_t)(ny - 1) * ny + kb]) : 0.f;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            As[e / SG_KC][e % SG_KC] = ra[q];
            if (LEFT) Bs[e / BT][e % BT] = rb[q];
            else Bs[e % SG_KC][e / SG_KC] = rb[q];
        }
        if (erow && threadIdx.x < SG_KC) Ae[threadIdx.x] = rae;
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC) Be[threadIdx.x - 64] = rbe;
    };
    // DIVOUT: the eigenvalues and types of the tile's rows (LDS, ordered by the
    // chunk loop's first barrier) and of the thread's epilogue column
    // (threadIdx.x % BT), requested before the products; a type of 1 marks a
    // row or column outside the slice
    __shared__ double dv_sl[DIVOUT ? BT : 1];
    __shared__ int dv_st[DIVOUT ? BT : 1];
    double dv_c = 0.0;
    int dv_ct = 1;
    if (DIVOUT) {
        if (threadIdx.x < BT) {
            const int row = i0 + (int)threadIdx.x;
            dv_sl[threadIdx.x] = row < nx ? F.lx[fx * nx + row] : 0.0;
            dv_st[threadIdx.x] = row < nx ? F.tx[fx * nx + row] : 1;
        }
        const int col = j0 + (int)threadIdx.x % BT;
        if (col < ny) {
            dv_c = F.ly[fx * ny + col];
            dv_ct = F.ty[fx * ny + col];
        }
    }
    flt4 acc[WT][WT];
#pragma unroll
    for (int ti = 0; ti < WT; ++ti)
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) acc[ti][tj] = flt4{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += SG_KC) {
        stash();
        __syncthreads();
        if (k0 + SG_KC < K) fetch(k0 + SG_KC);
        if (MODE == 1) {
#pragma unroll
            for (int kk = 0; kk < SG_KC; kk += 4) {
                if (kk >= K - k0) break;            // the zero padding past K
                float av[WT], bv[WT];
#pragma unroll
                for (int ti = 0; ti < WT; ++ti) av[ti] = As[16 * (WT * wi + ti) + r16][kk + k4];
#pragma unroll
                for (int tj = 0; tj < WT; ++tj) bv[tj] = Bs[kk + k4][16 * (WT * wj + tj) + r16];
#pragma unroll
                for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < WT; ++tj)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kb = 0; kb < SG_KC; kb += 16) {
                if (kb >= K - k0) break;
                sht4 ahi[WT], amid[WT], bhi[WT], bmid[WT];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
#pragma unroll
                    for (int ti = 0; ti < WT; ++ti) {
                        short h, m;
                        split_bf16(As[16 * (WT * wi + ti) + r16][kb + 4 * k4 + e], h, m);
                        ahi[ti][e] = h;
                        amid[ti][e] = m;
                    }
#pragma unroll
                    for (int tj = 0; tj < WT; ++tj) {
                        short h, m;
                        split_bf16(Bs[kb + 4 * k4 + e][16 * (WT * wj + tj) + r16], h, m);
                        bhi[tj][e] = h;
                        bmid[tj][e] = m;
                    }
                }
#pragma unroll
                for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < WT; ++tj) {
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(amid[ti], bhi[tj], acc[ti][tj], 0, 0, 0);
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[ti], bmid[tj], acc[ti][tj], 0, 0, 0);
                        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[ti], bhi[tj], acc[ti][tj], 0, 0, 0);
                    }
            }
        }
        if (erow || ecol) {
            const int tx = threadIdx.x, kn = min(SG_KC, K - k0);
            if (erow && tx < BT)
                for (int kk = 0; kk < kn; ++kk) ext = fmaf(Ae[kk], Bs[kk][tx], ext);
            else if (ecol && tx >= BT && tx < 2 * BT)
                for (int kk = 0; kk < kn; ++kk) ext = fmaf(As[tx - BT][kk], Be[kk], ext);
            else if (erow && ecol && tx == 2 * BT)
                for (int kk = 0; kk < kn; ++kk) ext = fmaf(Ae[kk], Be[kk], ext);
        }
        __syncthreads();
    }
    // DIVOUT: an element (i, j) with real x and y eigenvalues divided by
    // lambda_x + lambda_y - E in FP64 as it is stored (complex pairs are
    // stored undivided for k_divide_pairs)
    auto divout = [&](int row, int col, float v) -> float {
        if (!DIVOUT) return v;
        const int ti = F.tx[fx * nx + row], tj = F.ty[fx * ny + col];
        if (ti != 0 || tj != 0) return v;
        return (float)((double)v * rcp_newton(F.lx[fx * nx + row] + F.ly[fx * ny + col] - E));
    };
    if (DIVOUT) {
        // the tile through LDS (the operand tiles are free after the last
        // barrier), then each thread divides and stores rows of one column
        // (rows padded to BT + 1)
        float *ot = sg32;
#pragma unroll
        for (int ti = 0; ti < WT; ++ti)
#pragma unroll
            for (int tj = 0; tj < WT; ++tj)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    ot[(16 * (WT * wi + ti) + 4 * k4 + v) * (BT + 1) + 16 * (WT * wj + tj) + r16] = acc[ti][tj][v];
        __syncthreads();
        const int c = (int)threadIdx.x % BT, col = j0 + c;
#pragma unroll 2
        for (int r = (int)threadIdx.x / BT; r < BT; r += 256 / BT) {
            const int row = i0 + r;
            if (row < nx && col < ny) {
                float val = ot[r * (BT + 1) + c];
                if ((dv_st[r] | dv_ct) == 0) val = (float)((double)val * rcp_newton(dv_sl[r] + dv_c - E));
                o[(size_t)row * ny + col] = (TO)val;
            }
        }
    } else {
#pragma unroll
        for (int ti = 0; ti < WT; ++ti)
#pragma unroll
            for (int tj = 0; tj < WT; ++tj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = i0 + 16 * (WT * wi + ti) + 4 * k4 + v, col = j0 + 16 * (WT * wj + tj) + r16;
                    if (row < nx && col < ny) o[(size_t)row * ny + col] = (TO)acc[ti][tj][v];
                }
    }
    if (erow || ecol) {
        const int tx = threadIdx.x;
        if (erow && tx < BT && j0 + tx < ny) o[(size_t)(nx - 1) * ny + j0 + tx] = (TO)divout(nx - 1, j0 + tx, ext);
        else if (ecol && tx >= BT && tx < 2 * BT && i0 + tx - BT < nx)
            o[(size_t)(i0 + tx - BT) * ny + ny - 1] = (TO)divout(i0 + tx - BT, ny - 1, ext);
        else if (erow && ecol && tx == 2 * BT) o[(size_t)(nx - 1) * ny + ny - 1] = (TO)divout(nx - 1, ny - 1, ext);
    }
}

// Staged x-y products in reduced precision (same tiling and pipelining as
// k_slice_gemm): MODE 1 FP32 MFMA, MODE 2 BF16x3 MFMA (each operand split into
// bfloat16 hi + mid on the fly, three products, FP32 sums).  Storage between
// the products stays FP64; DIV applies the FP64 divide while loading.
template <bool LEFT, bool DIV, int MODE>
__global__ void __launch_bounds__(256) k_slice_gemm_lp(const ProblemDev *__restrict__ pd,
                                                       const PrecDev *__restrict__ pr,
                                                       const double *__restrict__ Evec,
                                                       const int *__restrict__ active, int which,
                                                       const double *__restrict__ in, double *__restrict__ out) {
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    int a, iM, k;
    if (!slice_decode(pd, blockIdx.x, a, iM, k)) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nx = C.x.n, ny = C.y.n, nz = C.z.n;
    const int tc = sg_tiles(ny, SG_T);
    const int t = blockIdx.y;
    if (t >= sg_tiles(nx, SG_T) * tc) return;
    const int i0 = (t / tc) * SG_T, j0 = (t % tc) * SG_T;
    // the last tile of a side 32 m + 1 also computes line n - 1 (see sg_tiles)
    const bool erow = i0 + SG_T == nx - 1 && nx % SG_T == 1, ecol = j0 + SG_T == ny - 1 && ny % SG_T == 1;
    const size_t fx = (size_t)iM * nz + k;
    const float *Wm = LEFT ? F.Wx32 + (fx * 2 + which) * nx * nx : F.Wy32 + (fx * 2 + which) * ny * ny;
    const long long off = (long long)req * pd->N + C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    const double *g = in + off;
    double *o = out + off;
    const int K = LEFT ? nx : ny;
    const double E = DIV ? Evec[req] : 0.0;
    double mind = 1e300;
    __shared__ float As[SG_T][SG_KC + 1];   // [row][k]
    __shared__ float Bs[SG_KC][SG_T + 1];   // [k][col]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, k4 = lane >> 4, wi = wave >> 1, wj = wave & 1;
    constexpr int PER = SG_T * SG_KC / 256;
    float ra[PER], rb[PER];
    // leftover line (FP32 FMAs): A's row nx - 1 and B's column ny - 1 of the
    // chunk, loaded by threads 0..31 and 64..95; threads 0..31 sum the row
    // outputs, 32..63 the column outputs, 64 the corner
    __shared__ float Ae[SG_KC], Be[SG_KC];
    float rae = 0.f, rbe = 0.f, ext = 0.f;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int r = e / SG_KC, c = e % SG_KC;
            const int row = i0 + r, kk = k0 + c;
            float av = 0.f;
            if (row < nx && kk < K) av = LEFT ? Wm[(size_t)row * nx + kk] : (float)g[(size_t)row * ny + kk];
            ra[q] = av;
            float bv = 0.f;
            if (LEFT) {
                const int kb = e / SG_T, cb = e % SG_T;
                if (k0 + kb < K && j0 + cb < ny)
                    bv = (float)(DIV ? divided_at(g, ny, k0 + kb, j0 + cb, F.lx + fx * nx, F.lxi + fx * nx,
                                                  F.tx + fx * nx, F.ly + fx * ny, F.lyi + fx * ny, F.ty + fx * ny, E,
                                                  mind)
                                     : g[(size_t)(k0 + kb) * ny + j0 + cb]);
            } else {
                const int cb = e / SG_KC, kb = e % SG_KC;
                if (k0 + kb < K && j0 + cb < ny) bv = Wm[(size_t)(j0 + cb) * ny + k0 + kb];
            }
            rb[q] = bv;
        }
        if (erow && threadIdx.x < SG_KC) {
            const int kk = k0 + threadIdx.x;
            rae = kk < K ? (LEFT ? Wm[(size_t)(nx - 1) * nx + kk] : (float)g[(size_t)(nx - 1) * ny + kk]) : 0.f;
        }
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC) {
            const int kb = k0 + (int)threadIdx.x - 64;
            float bv = 0.f;
            if (kb < K) {
                if (!LEFT) bv = Wm[(size_t)(ny - 1) * ny + kb];
                else if (DIV) bv = (float)divided_at(g, ny, kb, ny - 1, F.lx + fx * nx, F.lxi + fx * nx, F.tx + fx * nx,
                                                     F.ly + fx * ny, F.lyi + fx * ny, F.ty + fx * ny, E, mind);
                else bv = (float)g[(size_t)kb * ny + ny - 1];
            }
            rbe = bv;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            As[e / SG_KC][e % SG_KC] = ra[q];
            if (LEFT) Bs[e / SG_T][e % SG_T] = rb[q];
            else Bs[e % SG_KC][e / SG_KC] = rb[q];
        }
        if (erow && threadIdx.x < SG_KC) Ae[threadIdx.x] = rae;
        if (ecol && threadIdx.x >= 64 && threadIdx.x < 64 + SG_KC) Be[threadIdx.x - 64] = rbe;
    };
    flt4 acc = flt4{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += SG_KC) {
        stash();
        __syncthreads();
        if (k0 + SG_KC < K) fetch(k0 + SG_KC);
        if (MODE == 1) {
#pragma unroll
            for (int kk = 0; kk < SG_KC; kk += 4) {
                if (kk >= K - k0) break;            // the zero padding past K
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(As[16 * wi + r16][kk + k4], Bs[kk + k4][16 * wj + r16], acc,
                                                           0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kb = 0; kb < SG_KC; kb += 16) {
                if (kb >= K - k0) break;
                sht4 ahi, amid, bhi, bmid;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    short h, m;
                    split_bf16(As[16 * wi + r16][kb + 4 * k4 + e], h, m);
                    ahi[e] = h;
                    amid[e] = m;
                    split_bf16(Bs[kb + 4 * k4 + e][16 * wj + r16], h, m);
                    bhi[e] = h;
                    bmid[e] = m;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(amid, bhi, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bmid, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
            }
        }
        if (erow || ecol) {
            const int tx = threadIdx.x, kn = min(SG_KC, K - k0);
            if (erow && tx < SG_T)
                for (int kk = 0; kk < kn; ++kk) ext = fmaf(Ae[kk], Bs[kk][tx], ext);
            else if (ecol && tx >= SG_T && tx < 2 * SG_T)
                for (int kk = 0; kk < kn; ++kk) ext = fmaf(As[tx - SG_T][kk], Be[kk], ext);
            else if (erow && ecol && tx == 2 * SG_T)
                for (int kk = 0; kk < kn; ++kk) ext = fmaf(Ae[kk], Be[kk], ext);
        }
        __syncthreads();
    }
    (void)mind;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = i0 + 16 * wi + 4 * k4 + v, col = j0 + 16 * wj + r16;
        if (row < nx && col < ny) o[(size_t)row * ny + col] = (double)acc[v];
    }
    if (erow || ecol) {
        const int tx = threadIdx.x;
        if (erow && tx < SG_T && j0 + tx < ny) o[(size_t)(nx - 1) * ny + j0 + tx] = (double)ext;
        else if (ecol && tx >= SG_T && tx < 2 * SG_T && i0 + tx - SG_T < nx)
            o[(size_t)(i0 + tx - SG_T) * ny + ny - 1] = (double)ext;
        else if (erow && ecol && tx == 2 * SG_T) o[(size_t)(nx - 1) * ny + ny - 1] = (double)ext;
    }
}

template <int MAXT, int MODE, int NW>
__global__ void __launch_bounds__(NW * 64) k_xy_lp(const ProblemDev *__restrict__ pd,
                                                      const PrecDev *__restrict__ pr,
                                                      const double *__restrict__ Evec,
                                                      const int *__restrict__ active, double *data) {
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    const int a = blockIdx.y / MAXM, iM = blockIdx.y % MAXM;
    if (iM >= pd->nM) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int k = blockIdx.x;
    const int nz = C.z.n, nx = C.x.n, ny = C.y.n;
    if (k >= nz) return;
    const int nxp = (nx + 15) & ~15, nyp = (ny + 15) & ~15, ld = nyp + 4;
    extern __shared__ float Tf[];
    double *g = data + (long long)req * pd->N + C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    for (int t = threadIdx.x; t < nxp * ld; t += NW * 64) {
        const int i = t / ld, j = t % ld;
        Tf[t] = (i < nx && j < ny) ? (float)g[i * ny + j] : 0.f;
    }
    __syncthreads();
    const size_t fx = (size_t)iM * nz + k;
    if (MODE == 1) {
        const float *Wbx = F.Wx32 + fx * 2 * nx * nx, *Wx = Wbx + (size_t)nx * nx;
        const float *Wby = F.Wy32 + fx * 2 * ny * ny, *Wy = Wby + (size_t)ny * ny;
        mfma32_slice_mult<true, MAXT, NW>(Tf, ld, nxp, nyp, Wbx, nx);
        mfma32_slice_mult<false, MAXT, NW>(Tf, ld, nxp, nyp, Wby, ny);
        block_divide_f32(Tf, ld, nx, ny, F.lx + fx * nx, F.lxi + fx * nx, F.tx + fx * nx, F.ly + fx * ny,
                         F.lyi + fx * ny, F.ty + fx * ny, Evec[req]);
        mfma32_slice_mult<true, MAXT, NW>(Tf, ld, nxp, nyp, Wx, nx);
        mfma32_slice_mult<false, MAXT, NW>(Tf, ld, nxp, nyp, Wy, ny);
    } else {
        const size_t px = (size_t)pd->nM * nz * 2 * nx * nx, py = (size_t)pd->nM * nz * 2 * ny * ny;
        const unsigned short *Wbx = F.Wx16 + fx * 2 * nx * nx, *Wx = Wbx + (size_t)nx * nx;
        const unsigned short *Wby = F.Wy16 + fx * 2 * ny * ny, *Wy = Wby + (size_t)ny * ny;
        mfma_bf3_slice_mult<true, MAXT, NW>(Tf, ld, nxp, nyp, Wbx, px, nx);
        mfma_bf3_slice_mult<false, MAXT, NW>(Tf, ld, nxp, nyp, Wby, py, ny);
        block_divide_f32(Tf, ld, nx, ny, F.lx + fx * nx, F.lxi + fx * nx, F.tx + fx * nx, F.ly + fx * ny,
                         F.lyi + fx * ny, F.ty + fx * ny, Evec[req]);
        mfma_bf3_slice_mult<true, MAXT, NW>(Tf, ld, nxp, nyp, Wx, px, nx);
        mfma_bf3_slice_mult<false, MAXT, NW>(Tf, ld, nxp, nyp, Wy, py, ny);
    }
    for (int t = threadIdx.x; t < nx * ny; t += NW * 64) g[t] = (double)Tf[(t / ny) * ld + t % ny];
}

// Mode-z products in FP32 (the pass is bound by HBM traffic of FP64 vectors).
__global__ void __launch_bounds__(MZ_COLS) k_modez32(const ProblemDev *__restrict__ pd, const PrecDev *__restrict__ pr,
                                                     const int *__restrict__ active, int which, const double *in,
                                                     double *out) {
    const int req = blockIdx.z;
    if (active && !active[req]) return;
    const int a = blockIdx.y / MAXM, iM = blockIdx.y % MAXM;
    if (iM >= pd->nM) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nz = C.z.n, nxy = C.nxy;
    const int col0 = blockIdx.x * MZ_COLS;
    if (col0 >= nxy) return;
    extern __shared__ float smf[];
    float *W = smf;
    float *T = smf + nz * nz;
    const float *Wg = F.Wz32 + ((size_t)iM * 2 + which) * nz * nz;
    for (int t = threadIdx.x; t < nz * nz; t += MZ_COLS) W[t] = Wg[t];
    const long long base = (long long)req * pd->N + C.off + (long long)iM * C.npts;
    const int col = col0 + threadIdx.x;
    const bool ok = col < nxy;
    for (int k = 0; k < nz; ++k) T[k * MZ_COLS + threadIdx.x] = ok ? (float)in[base + (long long)k * nxy + col] : 0.f;
    __syncthreads();
    if (!ok) return;
    for (int k2 = 0; k2 < nz; ++k2) {
        float acc = 0;
        for (int k = 0; k < nz; ++k) acc += W[k2 * nz + k] * T[k * MZ_COLS + threadIdx.x];
        out[base + (long long)k2 * nxy + col] = (double)acc;
    }
}

// ---------------------------------------------------------------------------
// GMRES pieces.  V is stored [i][request][N]; Z likewise.
constexpr int RT = 256;              // threads of the reduction kernels
// two doubles as one 16-byte load or store (a clang vector type: the
// non-temporal builtins take it)
typedef double dv2 __attribute__((ext_vector_type(2)));
constexpr int MD_G = 8;              // vectors per group in the multi-dot

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block (NT threads); the result is valid in every thread.
template <int NT = RT>
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0;
    for (int wv = 0; wv < NT / 64; ++wv) r += red[wv];
    __syncthreads();
    return r;
}

// Returns true in the one block that arrives last for this request.
__device__ __forceinline__ bool last_block(unsigned *ticket, unsigned total) {
    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(ticket, 1u);
        last = (t == total - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

__device__ __forceinline__ void chunk_range(long long N, int blk, long long &lo, long long &hi) {
    long long per = (N + gridDim.x - 1) / gridDim.x;
    lo = blk * per;
    hi = min(N, lo + per);
}

// Sum of the n partials p[0..n) by the block; valid in every thread.
__device__ __forceinline__ double block_sum_parts(const double *__restrict__ p, int n, double *red) {
    double s = 0;
    for (int b = threadIdx.x; b < n; b += RT) s += p[b];
    return block_sum(s, red);
}

// Arnoldi with delayed reorthogonalisation (one dot pass and one update pass
// per step).  At step j the Krylov slots hold Q = v_0..v_{j-1} (orthonormal),
// U = v_j (the new direction, projected once against Q, not yet normalised) and
// W = v_{j+1} = A M^-1 U.  The dot pass forms s = Q^T U, t = Q^T W, U.U, U.W
// and W.W together; U then receives its second projection, q_j = (U - Q s) / r_j
// with r_j^2 = U.U - s.s, and W its first, (W - Q t - c_j q_j) / rho_j with
// c_j = q_j.W = (U.W - s.t) / r_j and rho_j^2 = W.W - t.t - c_j^2 (the norm of
// the projected W by Pythagoras; the scaling keeps the directions near unit
// length, so that their size does not grow or shrink step after step).  The
// Hessenberg column of step j - 1 is complete once s and r_j are known:
// h_{i,j-1} = t_i + rho_{j-1} s_i (with t_{j-1} = c_{j-1}) and
// h_{j,j-1} = rho_{j-1} r_j.  Since the preconditioner is applied to U,
// A M^-1 U is expressed in the orthonormal basis by exactly this column, and
// the solution update uses the stored M^-1 U directly.
//
// The basis vectors are read with non-temporal loads in both passes (each is
// streamed once per pass; measured 5-15 % faster than cached loads); U and W,
// which the next pass reads again, with ordinary ones.
// Dot pass partials, per block a row of 2m + 3 values: s_i at i, t_i at j + i,
// U.U at 2j, U.W at 2j + 1, W.W at 2j + 2.  CLOSING: no W (the last
// column of a cycle).
// Grid: (blocks per request, groups of G vectors of Q, requests); G = 4 or 8
// by j, so that few vector slots repeat.
template <bool CLOSING, int G>
__global__ void __launch_bounds__(RT) k_arnoldi_dots(KrylovDev K, int j) {
    constexpr int MD_G = G;
    const int req = blockIdx.z;
    if (!K.active[req]) return;
    __shared__ double red[2 * MD_G + 3][RT / 64];
    const int g0 = blockIdx.y * MD_G;
    const int ng = max(0, min(MD_G, j - g0));
    const bool lead = blockIdx.y == 0;
    long long lo, hi;
    chunk_range(K.N, blockIdx.x, lo, hi);
    const long long vstride = (long long)K.nb * K.N;
    const double *U = K.V + (long long)j * vstride + (long long)req * K.N;
    const double *W = U + vstride;
    const double *q0 = K.V + (long long)g0 * vstride + (long long)req * K.N;
    double as[MD_G], at[MD_G];
    double uu = 0, uw = 0, ww = 0;
#pragma unroll
    for (int t = 0; t < MD_G; ++t) as[t] = at[t] = 0;
    long long e = lo + threadIdx.x;
    if (ng > 0) {
        // U and W of this thread's elements (16 per chunk of the block) in
        // registers, then the group's vectors streamed one after another: one
        // basis vector in flight per wave at a time, as in the update pass.
        // With N and the block's chunk even, a thread's elements are pairs of
        // neighbours read with 16-byte loads; otherwise single elements.
        constexpr int EPT = 16;
        const long long per = (K.N + gridDim.x - 1) / gridDim.x;
        const bool pairs = (K.N & 1) == 0 && (per & 1) == 0;
        // element i of this thread in the chunk starting at e0
        auto elem = [&](long long e0, int i) {
            return pairs ? e0 + 2 * (long long)threadIdx.x + 2LL * RT * (i >> 1) + (i & 1)
                         : e0 + threadIdx.x + (long long)RT * i;
        };
        for (long long e0 = lo; e0 < hi; e0 += (long long)RT * EPT) {
            double u[EPT], w[EPT];
            if (pairs) {
#pragma unroll
                for (int i = 0; i < EPT; i += 2) {
                    const long long ee = elem(e0, i);
                    dv2 a = {0.0, 0.0}, b = {0.0, 0.0};
                    if (ee < hi) {
                        a = *reinterpret_cast<const dv2 *>(U + ee);
                        if (!CLOSING) b = *reinterpret_cast<const dv2 *>(W + ee);
                    }
                    u[i] = a.x;
                    u[i + 1] = a.y;
                    w[i] = b.x;
                    w[i + 1] = b.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    const long long ee = elem(e0, i);
                    u[i] = ee < hi ? U[ee] : 0.0;
                    w[i] = (!CLOSING && ee < hi) ? W[ee] : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                uu += u[i] * u[i];
                uw += u[i] * w[i];
                ww += w[i] * w[i];
            }
#pragma unroll
            for (int t = 0; t < MD_G; ++t)
                if (t < ng) {
                    const double *q = q0 + (long long)t * vstride;
                    double qa[EPT];
                    if (pairs) {
#pragma unroll
                        for (int i = 0; i < EPT; i += 2) {
                            const long long ee = elem(e0, i);
                            dv2 a = {0.0, 0.0};
                            if (ee < hi) a = __builtin_nontemporal_load(reinterpret_cast<const dv2 *>(q + ee));
                            qa[i] = a.x;
                            qa[i + 1] = a.y;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < EPT; ++i) {
                            const long long ee = elem(e0, i);
                            qa[i] = ee < hi ? __builtin_nontemporal_load(q + ee) : 0.0;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < EPT; ++i) {
                        as[t] += qa[i] * u[i];
                        if (!CLOSING) at[t] += qa[i] * w[i];
                    }
                }
        }
    } else {
        for (; e < hi; e += RT) {
            const double u0 = U[e], w0 = CLOSING ? 0.0 : W[e];
            uu += u0 * u0;
            uw += u0 * w0;
            ww += w0 * w0;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < MD_G; ++t)
        if (t < ng) {
            const double a = wave_sum(as[t]), b = wave_sum(at[t]);
            if (lane == 0) {
                red[t][wave] = a;
                red[MD_G + t][wave] = b;
            }
        }
    if (lead) {
        const double a = wave_sum(uu), b = wave_sum(uw), c = wave_sum(ww);
        if (lane == 0) {
            red[2 * MD_G][wave] = a;
            red[2 * MD_G + 1][wave] = b;
            red[2 * MD_G + 2][wave] = c;
        }
    }
    __syncthreads();
    // partials block-major: part[block][row], row stride 2m + 3
    double *part = K.part + (size_t)req * (2 * K.m + 3) * NBLK + (size_t)blockIdx.x * (2 * K.m + 3);
    const int r = threadIdx.x;
    int row = -1;
    if (r < ng) row = g0 + r;
    else if (r >= MD_G && r < MD_G + ng) row = j + g0 + (r - MD_G);
    else if (lead && r == 2 * MD_G) row = 2 * j;
    else if (lead && r == 2 * MD_G + 1) row = 2 * j + 1;
    else if (lead && r == 2 * MD_G + 2) row = 2 * j + 2;
    if (row >= 0) {
        double s = 0;
        for (int wv = 0; wv < RT / 64; ++wv) s += red[r][wv];
        part[row] = s;
    }
}

constexpr int FT = 1024;             // threads of the step-completion kernel (its waves split the blocks' partials)

// Completes step j of every active request from the dot-pass partials: s, t,
// r_j by Pythagoras (r_j = 0 when U.U - s.s is below 1e-20 U.U: U lies in the
// span of Q), the Hessenberg column j - 1 with its Givens rotation and the
// residual estimate |g_j|; a request leaves the cycle when that estimate meets
// its tolerance, on breakdown, or when closing.  Otherwise stores s (hproj),
// t and c_j (hcol), r_j (scal) and rho_j (rho; at least 1e-8 |W|, and 1 for
// W = 0) for the update pass.  rho holds rho_{j-1} on entry (for j = 0 the
// norm of the residual that v_0 was scaled by).  One block per request.
__global__ void __launch_bounds__(FT) k_arnoldi_finish(KrylovDev K, int j, int nblk, int closing) {
    const int req = blockIdx.x;
    if (!K.active[req]) return;
    __shared__ double sv[MAX_RESTART + 1], tv[MAX_RESTART + 1], col[MAX_RESTART + 1];
    __shared__ double csv[MAX_RESTART], snv[MAX_RESTART];
    __shared__ double red[FT / 64], uu_uw[3];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = K.m;
    const double *part = K.part + (size_t)req * (2 * m + 3) * NBLK;
    // the step's other inputs, requested now so that they arrive while the
    // partials are summed (the row loop's barriers publish the LDS copies)
    double *hc = K.hcol + (size_t)req * (m + 1);
    double *cs = K.cs + (size_t)req * m, *sn = K.sn + (size_t)req * m;
    double *g = K.g + (size_t)req * (m + 1);
    const double rho = K.rho[req];
    double g_prev = 0.0, tol = 0.0;
    if (threadIdx.x == 0 && j > 0) {
        g_prev = g[j - 1];
        tol = K.tol[req];
    }
    for (int i = threadIdx.x; i < j; i += FT) col[i] = hc[i];
    for (int i = threadIdx.x; i + 1 < j; i += FT) {
        csv[i] = cs[i];
        snv[i] = sn[i];
    }
    // row sums of the partials, 64 rows at a time: lane = row, the waves split
    // the blocks (fixed assignment, so the sums are deterministic); each wave
    // requests up to ILP of its blocks' values at once
    __shared__ double rsum[FT / 64][64];
    const int nrows = 2 * j + 3;
    for (int r0 = 0; r0 < nrows; r0 += 64) {
        const int row = r0 + lane;
        constexpr int NW = FT / 64, ILP = 8;
        double a[ILP];
#pragma unroll
        for (int u = 0; u < ILP; ++u) a[u] = 0;
        if (row < nrows) {
            const size_t rs = 2 * m + 3;
            for (int b = wave; b < nblk; b += ILP * NW) {
                double v[ILP];
#pragma unroll
                for (int u = 0; u < ILP; ++u) v[u] = b + u * NW < nblk ? part[(size_t)(b + u * NW) * rs + row] : 0.0;
#pragma unroll
                for (int u = 0; u < ILP; ++u) a[u] += v[u];
            }
        }
        double tot = 0;
#pragma unroll
        for (int u = 0; u < ILP; ++u) tot += a[u];
        rsum[wave][lane] = tot;
        __syncthreads();
        if (wave == 0 && row < nrows) {
            double s = 0;
            for (int w = 0; w < FT / 64; ++w) s += rsum[w][lane];
            if (row < j) sv[row] = s;
            else if (row < 2 * j) tv[row - j] = s;
            else uu_uw[row - 2 * j] = s;
        }
        __syncthreads();
    }
    double ss = 0, st = 0, tt = 0;
    for (int i = threadIdx.x; i < j; i += FT) {
        ss += sv[i] * sv[i];
        st += sv[i] * tv[i];
        tt += tv[i] * tv[i];
        col[i] += rho * sv[i];
    }
    ss = block_sum<FT>(ss, red);
    st = block_sum<FT>(st, red);
    tt = block_sum<FT>(tt, red);
    const double uu = uu_uw[0], uw = uu_uw[1], ww = uu_uw[2];
    const double r2 = uu - ss;
    const double r = (r2 > 1e-20 * uu) ? sqrt(r2) : 0.0;
    if (threadIdx.x == 0) {
        bool stop = closing != 0 || r == 0.0;
        if (j == 0) {
            g[0] = rho * r;
        } else {
            double *H = K.H + (size_t)req * (m + 1) * m;
            double carry = col[0];
            for (int i = 0; i + 1 < j; ++i) {
                const double b = col[i + 1], c = csv[i], s = snv[i];
                H[(size_t)i * m + (j - 1)] = c * carry + s * b;
                carry = -s * carry + c * b;
            }
            const double rr = hypot(carry, rho * r);
            const double c = rr > 0 ? carry / rr : 1.0, s = rr > 0 ? rho * r / rr : 0.0;
            cs[j - 1] = c;
            sn[j - 1] = s;
            H[(size_t)(j - 1) * m + (j - 1)] = rr;
            const double gj = -s * g_prev;
            g[j] = gj;
            g[j - 1] = c * g_prev;
            const double est = fabs(gj);
            if (!(est == est) || !(rr == rr)) {
                K.flags[req] |= 2;
                stop = true;
            }
            if (est <= tol) stop = true;
        }
        K.jcount[req] = j;
        if (!(r == r)) {
            K.flags[req] |= 2;
            stop = true;
        }
        if (closing) K.closed[req] = 1;
        if (stop) K.active[req] = 0;
        else K.scal[req] = r;
        red[0] = stop ? 1.0 : 0.0;
    }
    __syncthreads();
    if (red[0] != 0.0) return;
    double *hp = K.hproj + (size_t)req * (m + 1);
    for (int i = threadIdx.x; i < j; i += FT) {
        hp[i] = sv[i];
        hc[i] = tv[i];
    }
    if (threadIdx.x == 0) {
        const double c = (uw - st) / r;
        hc[j] = c;
        const double p2 = ww - tt - c * c;
        K.rho[req] = ww > 0 ? sqrt(fmax(p2, 1e-16 * ww)) : 1.0;
    }
}

// q_j = (U - Q s) / r_j over U and W = (W - Q t - c_j q_j) / rho_j, both in
// place: one pass over Q.  Dynamic LDS: s (j values) and t, c_j (j + 1 values).
__global__ void __launch_bounds__(RT) k_arnoldi_update(KrylovDev K, int j) {
    const int req = blockIdx.y;
    if (!K.active[req]) return;
    extern __shared__ double coef[];
    double *s = coef, *t = coef + j;
    const double *hp = K.hproj + (size_t)req * (K.m + 1), *hc = K.hcol + (size_t)req * (K.m + 1);
    for (int i = threadIdx.x; i < j; i += RT) s[i] = hp[i];
    for (int i = threadIdx.x; i <= j; i += RT) t[i] = hc[i];
    __syncthreads();
    const long long e = (long long)blockIdx.x * RT + threadIdx.x;
    if (e >= K.N) return;
    const long long vstride = (long long)K.nb * K.N;
    const double *q = K.V + (long long)req * K.N + e;
    double qs = 0, qt = 0;
    int i = 0;
    for (; i + 7 < j; i += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(q + (i + u) * vstride);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            qs += a[u] * s[i + u];
            qt += a[u] * t[i + u];
        }
    }
    for (; i < j; ++i) {
        const double a = __builtin_nontemporal_load(q + i * vstride);
        qs += a * s[i];
        qt += a * t[i];
    }
    double *U = K.V + (long long)j * vstride + (long long)req * K.N + e;
    double *W = U + vstride;
    const double inv = 1.0 / K.scal[req];
    const double qj = (*U - qs) * inv;
    *U = qj;
    *W = (*W - qt - t[j] * qj) * (1.0 / K.rho[req]);
}

// Two adjacent elements per thread with 16-byte loads and stores (N even, so
// that every vector of the basis starts on a 16-byte boundary).
__global__ void __launch_bounds__(RT) k_arnoldi_update2(KrylovDev K, int j) {
    const int req = blockIdx.y;
    if (!K.active[req]) return;
    extern __shared__ double coef[];
    double *s = coef, *t = coef + j;
    const double *hp = K.hproj + (size_t)req * (K.m + 1), *hc = K.hcol + (size_t)req * (K.m + 1);
    for (int i = threadIdx.x; i < j; i += RT) s[i] = hp[i];
    for (int i = threadIdx.x; i <= j; i += RT) t[i] = hc[i];
    __syncthreads();
    const long long e = 2 * ((long long)blockIdx.x * RT + threadIdx.x);
    if (e >= K.N) return;
    const long long vstride = (long long)K.nb * K.N;
    const dv2 *q = reinterpret_cast<const dv2 *>(K.V + (long long)req * K.N + e);
    const long long vs2 = vstride / 2;
    double qs0 = 0, qt0 = 0, qs1 = 0, qt1 = 0;
    int i = 0;
    for (; i + 7 < j; i += 8) {
        dv2 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(q + (i + u) * vs2);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            qs0 += a[u].x * s[i + u];
            qt0 += a[u].x * t[i + u];
            qs1 += a[u].y * s[i + u];
            qt1 += a[u].y * t[i + u];
        }
    }
    for (; i < j; ++i) {
        const dv2 a = __builtin_nontemporal_load(q + i * vs2);
        qs0 += a.x * s[i];
        qt0 += a.x * t[i];
        qs1 += a.y * s[i];
        qt1 += a.y * t[i];
    }
    dv2 *U = reinterpret_cast<dv2 *>(K.V + (long long)j * vstride + (long long)req * K.N + e);
    dv2 *W = U + vs2;
    const double inv = 1.0 / K.scal[req], rinv = 1.0 / K.rho[req];
    const dv2 u = *U, w = *W;
    dv2 qj, wn;
    qj.x = (u.x - qs0) * inv;
    qj.y = (u.y - qs1) * inv;
    wn.x = (w.x - qt0 - t[j] * qj.x) * rinv;
    wn.y = (w.y - qt1 - t[j] * qj.y) * rinv;
    *U = qj;
    *W = wn;
}

// y = R^-1 g for the steps of this cycle, one block per request, by columns:
// once y_i is known, every row above it takes its column-i term at once (the
// block's threads share the rows), so a step costs one barrier; each thread
// reads its rows of the next column while the current one is applied.
constexpr int CS_ROWS = (MAX_RESTART + RT - 1) / RT;   // rows per thread
__global__ void __launch_bounds__(RT) k_cycle_solve(KrylovDev K, const int *__restrict__ running) {
    const int req = blockIdx.x;
    if (!running[req]) return;
    const int m = K.m, jc = K.jcount[req];
    const double *H = K.H + (size_t)req * (m + 1) * m;
    const double *g = K.g + (size_t)req * (m + 1);
    double *y = K.y + (size_t)req * m;
    __shared__ double yi[2];
    double r[CS_ROWS], h[CS_ROWS], dg[CS_ROWS];
#pragma unroll
    for (int k = 0; k < CS_ROWS; ++k) {
        const int row = threadIdx.x + RT * k;
        r[k] = row < jc ? g[row] : 0.0;
        dg[k] = row < jc ? H[(size_t)row * m + row] : 0.0;
        h[k] = row < jc - 1 ? H[(size_t)row * m + (jc - 1)] : 0.0;
    }
    for (int i = jc - 1; i >= 0; --i) {
        // the owner of row i finishes it
        if ((i % RT) == (int)threadIdx.x) {
            const int k = i / RT;
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < CS_ROWS; ++u)
                if (u == k) v = dg[u] != 0.0 ? r[u] / dg[u] : 0.0;
            y[i] = v;
            yi[i & 1] = v;
        }
        __syncthreads();
        const double v = yi[i & 1];
        double hn[CS_ROWS];
#pragma unroll
        for (int k = 0; k < CS_ROWS; ++k) {
            const int row = threadIdx.x + RT * k;
            hn[k] = (i > 0 && row < i - 1) ? H[(size_t)row * m + (i - 1)] : 0.0;
            if (row < i) r[k] -= h[k] * v;
            h[k] = hn[k];
        }
    }
}

// x += sum_i z_i y_i
__global__ void __launch_bounds__(RT) k_xupdate(KrylovDev K, const int *__restrict__ running, double *X) {
    const int req = blockIdx.y;
    if (!running[req]) return;
    const int jc = K.jcount[req];
    __shared__ double y[1024];
    for (int i = threadIdx.x; i < jc; i += RT) y[i] = K.y[(size_t)req * K.m + i];
    __syncthreads();
    long long e = (long long)blockIdx.x * RT + threadIdx.x;
    if (e >= K.N) return;
    double acc = X[(long long)req * K.N + e];
    for (int i = 0; i < jc; ++i) acc += __builtin_nontemporal_load(K.Z + ((long long)i * K.nb + req) * K.N + e) * y[i];
    X[(long long)req * K.N + e] = acc;
}

// r = b - Ax into V slot 0, ||r||; then restart state or completion.
__global__ void __launch_bounds__(RT) k_residual(KrylovDev K, int *running, const double *__restrict__ B,
                                                 double rtol, double inner_safety) {
    const int req = blockIdx.y;
    if (!running[req]) return;
    __shared__ double red[RT];
    long long lo, hi;
    chunk_range(K.N, blockIdx.x, lo, hi);
    double *r = K.V + (long long)req * K.N;        // slot 0 holds A x on entry
    const double *b = B + (long long)req * K.N;
    double acc = 0;
    for (long long e = lo + threadIdx.x; e < hi; e += RT) {
        double v = b[e] - r[e];
        r[e] = v;
        acc += v * v;
    }
    double s = block_sum(acc, red);
    double *part = K.part + (size_t)req * (2 * K.m + 3) * NBLK;
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(&K.ticket[req], gridDim.x)) {
        const double rn = sqrt(block_sum_parts(part, gridDim.x, red));
        double *g = K.g + (size_t)req * (K.m + 1);
        for (int i = threadIdx.x; i <= K.m; i += RT) g[i] = i == 0 ? rn : 0.0;
        if (threadIdx.x == 0) {
            K.rnorm[req] = rn;
            K.rho[req] = rn;
            K.jcount[req] = 0;
            K.closed[req] = 0;
            if (!(rn == rn)) {
                K.flags[req] |= 2;
                running[req] = 0;
                K.active[req] = 0;
            } else if (rn <= rtol * K.bnorm[req] || rn == 0.0) {
                running[req] = 0;
                K.active[req] = 0;
            } else {
                K.active[req] = 1;
                K.tol[req] = inner_safety * rtol * K.bnorm[req];
            }
            K.ticket[req] = 0;
        }
    }
}

// v_0 = r / ||r|| for the requests that go on.
__global__ void __launch_bounds__(RT) k_scale0(KrylovDev K) {
    const int req = blockIdx.y;
    if (!K.active[req]) return;
    const long long e = (long long)blockIdx.x * RT + threadIdx.x;
    if (e >= K.N) return;
    double *v = K.V + (long long)req * K.N;
    v[e] = v[e] / K.rho[req];
}

__global__ void __launch_bounds__(RT) k_bnorm(KrylovDev K, const double *__restrict__ B, const int *__restrict__ mask) {
    const int req = blockIdx.y;
    if (mask && !mask[req]) return;
    __shared__ double red[RT];
    long long lo, hi;
    chunk_range(K.N, blockIdx.x, lo, hi);
    const double *b = B + (long long)req * K.N;
    double acc = 0;
    int bad = 0;
    for (long long e = lo + threadIdx.x; e < hi; e += RT) {
        double v = b[e];
        if (!(v - v == 0.0)) bad = 1;
        acc += v * v;
    }
    double s = block_sum(acc, red);
    __shared__ int anybad;
    if (threadIdx.x == 0) anybad = 0;
    __syncthreads();
    if (bad) atomicOr(&anybad, 1);
    __syncthreads();
    double *part = K.part + (size_t)req * (2 * K.m + 3) * NBLK;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        if (anybad) atomicOr(&K.flags[req], 1);
    }
    if (last_block(&K.ticket[req], gridDim.x)) {
        const double nn = block_sum_parts(part, gridDim.x, red);
        if (threadIdx.x == 0) {
            K.bnorm[req] = sqrt(nn);
            K.ticket[req] = 0;
        }
    }
}

// x = 0 and A x = 0 (Krylov slot 0) for the masked requests.
__global__ void k_zero_start(KrylovDev K, double *X, const int *__restrict__ mask, int zero_x) {
    const int req = blockIdx.y;
    if (!mask[req]) return;
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K.N) return;
    if (zero_x) X[(long long)req * K.N + e] = 0.0;
    K.V[(long long)req * K.N + e] = 0.0;
}

__global__ void k_fill(double *p, long long n, double v) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void k_copy(double *d, const double *__restrict__ s, long long n) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) d[e] = s[e];
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

template <int QXY, int QZ, int NM>
void launch_tiled(const ProblemDev &pd, int nb, const double *E_dev, const int *active, const double *x, double *y,
                  double *cbuf, hipStream_t st, int part) {
    if (part != 1 && pd.cpl.njobs > 0) {
        dim3 grid(cdiv(pd.cpl.njobs, CPL_WAVES), cdiv(nb, CPL_REQ));
        if (NM == 1 && pd.cpl.pairs_per_lane == 2)
            hipLaunchKernelGGL((k_coupling_cells<QXY, QZ, NM, NM == 1 ? 2 : 1>), grid, dim3(64 * CPL_WAVES), 0, st, pd.dev,
                               active, nb, x, cbuf);
        else
            hipLaunchKernelGGL((k_coupling_cells<QXY, QZ, NM, 1>), grid, dim3(64 * CPL_WAVES), 0, st, pd.dev, active, nb, x,
                               cbuf);
    }
    if (part != 2) {
        // tile counts padded to a multiple of 8 (XCD-aware tile order)
        if (NM == 1) {
            const unsigned tiles = (pd.comp[0].ntiles_g + pd.comp[1].ntiles_g + pd.comp[2].ntiles_g + 7) & ~7u;
            hipLaunchKernelGGL((k_local_grouped<QXY, QXY, QZ>), dim3(tiles, nb), dim3(256),
                               sizeof(double) * pd.group_lds, st, pd.dev, E_dev, active, x, y, cbuf);
        } else {
            const unsigned tiles = (pd.comp[0].ntiles + pd.comp[1].ntiles + pd.comp[2].ntiles + 7) & ~7u;
            hipLaunchKernelGGL((k_local_tiled<QXY, QXY, QZ, NM>), dim3(tiles, nb), dim3(256),
                               sizeof(double) * pd.plane_lds, st, pd.dev, E_dev, active, x, y, cbuf, nb);
        }
    }
}

// More M' blocks (n_M > 3): the coupling and local kernels that take the
// blocks one at a time.
template <int QXY, int QZ>
void launch_many(const ProblemDev &pd, int nb, const double *E_dev, const int *active, const double *x, double *y,
                 double *cbuf, hipStream_t st, int part) {
    if (part != 1 && pd.cpl.njobs > 0) {
        dim3 grid(cdiv(pd.cpl.njobs, CPL_WAVES), cdiv(nb, CPL_REQ));
        hipLaunchKernelGGL((k_coupling_many<QXY, QZ>), grid, dim3(64 * CPL_WAVES), 0, st, pd.dev, active, nb, x, cbuf);
    }
    if (part != 2) {
        const unsigned tiles = (pd.comp[0].ntiles + pd.comp[1].ntiles + pd.comp[2].ntiles + 7) & ~7u;
        hipLaunchKernelGGL((k_local_many<QXY, QXY, QZ>), dim3(tiles, nb), dim3(256), sizeof(double) * pd.plane_lds, st,
                           pd.dev, E_dev, active, x, y, cbuf);
    }
}

void launch_matvec(const ProblemDev &pd, int nb, const double *E_dev, const int *active, const double *x, double *y,
                   double *cbuf, hipStream_t st, int part) {
    if (matvec_tiled_ok(pd) && pd.nM > 3) {
        switch ((pd.q[0] == 3 ? 2 : 0) + (pd.q[2] == 3 ? 1 : 0)) {
            case 3: launch_many<3, 3>(pd, nb, E_dev, active, x, y, cbuf, st, part); return;
            case 2: launch_many<3, 2>(pd, nb, E_dev, active, x, y, cbuf, st, part); return;
            case 1: launch_many<2, 3>(pd, nb, E_dev, active, x, y, cbuf, st, part); return;
            default: launch_many<2, 2>(pd, nb, E_dev, active, x, y, cbuf, st, part); return;
        }
    }
    if (matvec_tiled_ok(pd)) {
        const int key = (pd.q[0] == 3 ? 4 : 0) + (pd.q[2] == 3 ? 2 : 0);
        switch (key * 4 + pd.nM) {
#define FM_TILED(QXY, QZ, NM) \
    case ((QXY == 3 ? 4 : 0) + (QZ == 3 ? 2 : 0)) * 4 + NM: launch_tiled<QXY, QZ, NM>(pd, nb, E_dev, active, x, y, cbuf, st, part); return;
            FM_TILED(3, 3, 1) FM_TILED(3, 3, 2) FM_TILED(3, 3, 3)
            FM_TILED(3, 2, 1) FM_TILED(3, 2, 2) FM_TILED(3, 2, 3)
            FM_TILED(2, 3, 1) FM_TILED(2, 3, 2) FM_TILED(2, 3, 3)
            FM_TILED(2, 2, 1) FM_TILED(2, 2, 2) FM_TILED(2, 2, 3)
#undef FM_TILED
            default: break;
        }
    }
    if (part == 2) return;            // the generic kernel computes the coupling with the rest
    long long pts = pd.comp[0].npts + pd.comp[1].npts + pd.comp[2].npts;
    dim3 grid(cdiv(pts, 256), nb);
    hipLaunchKernelGGL(k_matvec, grid, dim3(256), 0, st, pd.dev, E_dev, active, x, y);
}

// Launches the register-column mode-z kernel for nz <= 64, else the LDS one.
template <bool F32, class TI = double, class TO = double>
bool launch_modez_reg(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which,
                      const TI *in, TO *out, hipStream_t st) {
    int maxnxy = 0, maxnz = 0;
    for (int a = 0; a < 3; ++a) {
        maxnxy = std::max(maxnxy, pd.comp[a].nxy);
        maxnz = std::max(maxnz, pd.comp[a].z.n);
    }
    // split a column's outputs over up to 8 threads until the launch has about
    // 256 K threads (at most as many groups of four outputs as there are); a
    // launch of 256-512 K columns still gains from two threads per column
    // (measured 23 -> 21 us at 393 K columns), a larger split does not
    const long long cols = (long long)maxnxy * 3 * pd.nM * nb;
    int split = 1;
    while (split < 8 && 4 * split < maxnz && cols * split < 256 * 1024) split *= 2;
    if (split == 1 && 4 < maxnz && cols < 512 * 1024) split = 2;
    dim3 grid(cdiv(maxnxy, MZ2_THREADS / split), 3 * pd.nM, nb);
#define FM_MZ(M) hipLaunchKernelGGL((k_modez_reg<M, F32, TI, TO>), grid, dim3(MZ2_THREADS), 0, st, pd.dev, pr.dev, active, which, in, out, split)
    if (maxnz <= 16) FM_MZ(16);
    else if (maxnz <= 32) FM_MZ(32);
    else if (maxnz <= 48) FM_MZ(48);
    else if (maxnz <= 64) FM_MZ(64);
    else return false;
#undef FM_MZ
    return true;
}

void launch_modez(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which, const double *in,
                  double *out, hipStream_t st) {
    if (launch_modez_reg<false>(pd, pr, nb, active, which, in, out, st)) return;
    int maxnxy = 0, maxnz = 0;
    for (int a = 0; a < 3; ++a) {
        maxnxy = std::max(maxnxy, pd.comp[a].nxy);
        maxnz = std::max(maxnz, pd.comp[a].z.n);
    }
    dim3 grid(cdiv(maxnxy, MZ_COLS), 3 * MAXM, nb);
    size_t sh = sizeof(double) * (maxnz * maxnz + maxnz * MZ_COLS);
    hipLaunchKernelGGL(k_modez, grid, dim3(MZ_COLS), sh, st, pd.dev, pr.dev, active, which, in, out);
}

// Coupled preconditioner: out = Z in per component with its joint z matrix
// (which: 0 forward, 1 backward); in and out must not overlap.
void launch_zjoint(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which, const double *in,
                   double *out, hipStream_t st) {
    int tiles = 0;
    for (int a = 0; a < 3; ++a)
        tiles = std::max(tiles, (int)(cdiv(pd.nM * pd.comp[a].z.n, 64) * cdiv(pd.comp[a].nxy, 64)));
    const dim3 g(tiles, 3, nb);
    hipLaunchKernelGGL((k_slice_gemm<true, false, true, 64>), g, dim3(256), 0, st, pd.dev, pr.dev, nullptr, active,
                       which, in, out, nullptr);
}

void launch_xy(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active, double *data,
               double *min_den, double *tmp, hipStream_t st) {
    int slices = 0, tiles = 0, side = 0;
    for (int a = 0; a < 3; ++a) {
        slices += pd.nM * pd.comp[a].z.n;
        tiles = std::max(tiles, (int)(cdiv(pd.comp[a].x.n, SG_T) * cdiv(pd.comp[a].y.n, SG_T)));
        side = std::max(side, std::max(pd.comp[a].x.n, pd.comp[a].y.n));
    }
    if (side > XY_FUSED_MAX_SIDE) {
        // 64 x 64 block tiles (2 x 2 MFMA tiles per wave) for slices wider than 32
#define FM_SG(BT)                                                                                                      \
    {                                                                                                                  \
        int tl = 0;                                                                                                    \
        for (int a = 0; a < 3; ++a)                                                                                    \
            tl = std::max(tl, sg_tiles(pd.comp[a].x.n, BT) * sg_tiles(pd.comp[a].y.n, BT));                             \
        const dim3 g(slices, tl, nb);                                                                                  \
        hipLaunchKernelGGL((k_slice_gemm<true, false, false, BT>), g, dim3(256), 0, st, pd.dev, pr.dev, E_dev, active, \
                           0, data, tmp, nullptr);                                                                     \
        hipLaunchKernelGGL((k_slice_gemm<false, false, false, BT, true>), g, dim3(256), 0, st, pd.dev, pr.dev, E_dev,  \
                           active, 0, tmp, data, min_den);                                                             \
        if (pr.npair_slices > 0)                                                                                       \
            hipLaunchKernelGGL(k_divide_pairs<double>, dim3(pr.npair_slices, nb), dim3(256), 0, st, pd.dev, pr.dev, E_dev,     \
                               active, data, min_den);                                                                 \
        hipLaunchKernelGGL((k_slice_gemm<true, false, false, BT>), g, dim3(256), 0, st, pd.dev, pr.dev, E_dev, active, \
                           1, data, tmp, nullptr);                                                                     \
        hipLaunchKernelGGL((k_slice_gemm<false, false, false, BT>), g, dim3(256), 0, st, pd.dev, pr.dev, E_dev,        \
                           active, 1, tmp, data, nullptr);                                                             \
    }
        // 64 x 64 tiles reuse each operand chunk twice as often, but a small
        // batch of wide slices then leaves the chip short of blocks, and a side
        // of 32 m + 1 pads to far more area in 64-wide tiles than in 32-wide
        // ones with the leftover line (97: 128^2 against 96^2 + a line)
        long long t64 = 0, area64 = 0, area32 = 0;
        for (int a = 0; a < 3; ++a) {
            const int nx = pd.comp[a].x.n, ny = pd.comp[a].y.n;
            t64 = std::max<long long>(t64, (long long)sg_tiles(nx, 64) * sg_tiles(ny, 64));
            area64 += 4096LL * sg_tiles(nx, 64) * sg_tiles(ny, 64);
            area32 += 1024LL * sg_tiles(nx, 32) * sg_tiles(ny, 32);
        }
        if (side > 32 && t64 * slices * nb >= XY_T64_MIN_BLOCKS && 4 * area64 <= 5 * area32) FM_SG(64) else FM_SG(32)
#undef FM_SG
        (void)tiles;
        return;
    }
    // many slices of side <= 32: one block per slice, one 16 x 16 output tile per wave
    int maxnz = 0;
    size_t shm = 0;
    for (int a = 0; a < 3; ++a) {
        maxnz = std::max(maxnz, pd.comp[a].z.n);
        const int nxp = (pd.comp[a].x.n + 15) & ~15, nyp = (pd.comp[a].y.n + 15) & ~15;
        shm = std::max(shm, sizeof(double) * nxp * (nyp + 4));
    }
    dim3 grid(maxnz, 3 * MAXM, nb);
    hipLaunchKernelGGL((k_xy_mfma<1, 4>), grid, dim3(256), shm, st, pd.dev, pr.dev, E_dev, active, data, min_den);
}

void launch_modez_lp(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which, const double *in,
                     double *out, hipStream_t st) {
    if (launch_modez_reg<true>(pd, pr, nb, active, which, in, out, st)) return;
    int maxnxy = 0, maxnz = 0;
    for (int a = 0; a < 3; ++a) {
        maxnxy = std::max(maxnxy, pd.comp[a].nxy);
        maxnz = std::max(maxnz, pd.comp[a].z.n);
    }
    dim3 grid(cdiv(maxnxy, MZ_COLS), 3 * MAXM, nb);
    size_t sh = sizeof(float) * (maxnz * maxnz + maxnz * MZ_COLS);
    hipLaunchKernelGGL(k_modez32, grid, dim3(MZ_COLS), sh, st, pd.dev, pr.dev, active, which, in, out);
}

bool xy_lp_staged(const ProblemDev &pd, int nb, int mode);

bool launch_xy_lp(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active, double *data,
                  int mode, double *tmp, hipStream_t st) {
    {
        int slices = 0, tiles = 0, side = 0;
        for (int a = 0; a < 3; ++a) {
            slices += pd.nM * pd.comp[a].z.n;
            tiles = std::max(tiles, sg_tiles(pd.comp[a].x.n, SG_T) * sg_tiles(pd.comp[a].y.n, SG_T));
            side = std::max(side, std::max(pd.comp[a].x.n, pd.comp[a].y.n));
        }
        if (xy_lp_staged(pd, nb, mode)) {
            const dim3 g(slices, tiles, nb);
#define FM_SGLP(L, D, M, W, I, O) \
    hipLaunchKernelGGL((k_slice_gemm_lp<L, D, M>), g, dim3(256), 0, st, pd.dev, pr.dev, E_dev, active, W, I, O)
            if (mode == 1) {
                FM_SGLP(true, false, 1, 0, data, tmp);
                FM_SGLP(false, false, 1, 0, tmp, data);
                FM_SGLP(true, true, 1, 1, data, tmp);
                FM_SGLP(false, false, 1, 1, tmp, data);
            } else {
                FM_SGLP(true, false, 2, 0, data, tmp);
                FM_SGLP(false, false, 2, 0, tmp, data);
                FM_SGLP(true, true, 2, 1, data, tmp);
                FM_SGLP(false, false, 2, 1, tmp, data);
            }
#undef FM_SGLP
            return true;
        }
    }
    int maxnz = 0, tpw = 0;
    size_t shm = 0;
    for (int a = 0; a < 3; ++a) {
        maxnz = std::max(maxnz, pd.comp[a].z.n);
        const int nxp = (pd.comp[a].x.n + 15) & ~15, nyp = (pd.comp[a].y.n + 15) & ~15;
        shm = std::max(shm, sizeof(float) * nxp * (nyp + 4));
        tpw = std::max(tpw, ((nxp / 16) * (nyp / 16) + 3) / 4);
    }
    if (tpw > XYM_MAXT || shm > xy_lds_limit()) return false;
    dim3 grid(maxnz, 3 * MAXM, nb);
#define FM_XYLP(T, NW)                                                                                         \
    {                                                                                                          \
        if (mode == 1) hipLaunchKernelGGL((k_xy_lp<T, 1, NW>), grid, dim3(NW * 64), shm, st, pd.dev, pr.dev, E_dev, active, data); \
        else hipLaunchKernelGGL((k_xy_lp<T, 2, NW>), grid, dim3(NW * 64), shm, st, pd.dev, pr.dev, E_dev, active, data); \
    }
    if (tpw <= 1) FM_XYLP(1, 4)
    else if (tpw <= 2) FM_XYLP(2, 4)
    else if (tpw <= 4) FM_XYLP(4, 4)
    else if (tpw <= 8) FM_XYLP(4, 8)
    else if (tpw <= 12) FM_XYLP(6, 8)
    else FM_XYLP(8, 8)
#undef FM_XYLP
    return true;
}

bool xy_lp_staged(const ProblemDev &pd, int nb, int mode) {
    long long slices = 0;
    int side = 0;
    for (int a = 0; a < 3; ++a) {
        slices += (long long)pd.nM * pd.comp[a].z.n;
        side = std::max(side, std::max(pd.comp[a].x.n, pd.comp[a].y.n));
    }
    // BF16x3 (three products per product) keeps the staged chain below
    // XY_BF16_FUSED_FROM slices, where its one-block-per-slice kernel is slower
    return side > XY_FUSED_MAX_SIDE || (mode == 2 && slices * nb < XY_BF16_FUSED_FROM);
}

// The four staged x-y products with FP32 storage between them: src (TI) ->
// A -> B -> A (with the FP64 divide) -> dst (TO); A and B: [nb][N] FP32.
template <int MODE, int BT, class TI, class TO>
void xy_f32_chain(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active,
                  const TI *src, float *A, float *B, TO *dst, hipStream_t st) {
    int slices = 0, tl = 0;
    for (int a = 0; a < 3; ++a) {
        slices += pd.nM * pd.comp[a].z.n;
        tl = std::max(tl, sg_tiles(pd.comp[a].x.n, BT) * sg_tiles(pd.comp[a].y.n, BT));
    }
    const dim3 g(slices, tl, nb);
    hipLaunchKernelGGL((k_slice_gemm_f32<true, MODE, BT, TI, float>), g, dim3(256), 0, st, pd.dev, pr.dev,
                       E_dev, active, 0, src, A);
    // the divide on the store of the second product (real eigenvalue pairs),
    // the complex-pair blocks in place after it, then a plain left product
    hipLaunchKernelGGL((k_slice_gemm_f32<false, MODE, BT, float, float, true>), g, dim3(256), 0, st, pd.dev,
                       pr.dev, E_dev, active, 0, A, B);
    if (pr.npair_slices > 0)
        hipLaunchKernelGGL(k_divide_pairs<float>, dim3(pr.npair_slices, nb), dim3(256), 0, st, pd.dev, pr.dev, E_dev,
                           active, B, (double *)nullptr);
    hipLaunchKernelGGL((k_slice_gemm_f32<true, MODE, BT, float, float>), g, dim3(256), 0, st, pd.dev, pr.dev,
                       E_dev, active, 1, B, A);
    hipLaunchKernelGGL((k_slice_gemm_f32<false, MODE, BT, float, TO>), g, dim3(256), 0, st, pd.dev, pr.dev,
                       E_dev, active, 1, A, dst);
}

template <class TI, class TO>
void xy_f32(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active, int mode,
            const TI *src, float *A, float *B, TO *dst, hipStream_t st) {
    int slices = 0, side = 0;
    long long t64 = 0, area64 = 0, area32 = 0;
    for (int a = 0; a < 3; ++a) {
        slices += pd.nM * pd.comp[a].z.n;
        const int nx = pd.comp[a].x.n, ny = pd.comp[a].y.n;
        side = std::max(side, std::max(nx, ny));
        t64 = std::max<long long>(t64, (long long)sg_tiles(nx, 64) * sg_tiles(ny, 64));
        area64 += 4096LL * sg_tiles(nx, 64) * sg_tiles(ny, 64);
        area32 += 1024LL * sg_tiles(nx, 32) * sg_tiles(ny, 32);
    }
    const bool t64ok = side > 32 && t64 * slices * nb >= XY_T64_MIN_BLOCKS && 4 * area64 <= 5 * area32;
    if (mode == 1) {
        if (t64ok) xy_f32_chain<1, 64>(pd, pr, nb, E_dev, active, src, A, B, dst, st);
        else xy_f32_chain<1, 32>(pd, pr, nb, E_dev, active, src, A, B, dst, st);
    } else {
        if (t64ok) xy_f32_chain<2, 64>(pd, pr, nb, E_dev, active, src, A, B, dst, st);
        else xy_f32_chain<2, 32>(pd, pr, nb, E_dev, active, src, A, B, dst, st);
    }
}

bool precond_f32_ok(const ProblemDev &pd, const PrecDev &pr, int nb, int mode) {
    if (!xy_lp_staged(pd, nb, mode)) return false;
    int maxnz = 0;
    for (int a = 0; a < 3; ++a) maxnz = std::max(maxnz, pd.comp[a].z.n);
    return pr.coupled || maxnz <= 64;
}

void launch_z_f32(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which, const double *in,
                  double *out, double *tmp, hipStream_t st) {
    float *B = reinterpret_cast<float *>(tmp);
    if (pr.coupled) {
        // the joint z products stay FP64 (as in every variant)
        if (which == 0) launch_zjoint(pd, pr, nb, active, 0, in, tmp, st);
        else launch_zjoint(pd, pr, nb, active, 1, tmp, out, st);
        return;
    }
    if (which == 0) launch_modez_reg<true, double, float>(pd, pr, nb, active, 0, in, B, st);
    else launch_modez_reg<true, float, double>(pd, pr, nb, active, 1, B, out, st);
}

void launch_xy_f32(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active, int mode,
                   double *out, double *tmp, hipStream_t st) {
    float *A = reinterpret_cast<float *>(out), *B = reinterpret_cast<float *>(tmp);
    if (pr.coupled) xy_f32<double, double>(pd, pr, nb, E_dev, active, mode, tmp, A, B, tmp, st);
    else xy_f32<float, float>(pd, pr, nb, E_dev, active, mode, B, A, B, B, st);
}

// Groups of 8 vectors: as fast as 16 while every request iterates, and faster
// once few are left (twice the blocks per request).
int dots_group(int j) { return j <= 4 ? 4 : MD_G; }

unsigned dots_blocks(const KrylovDev &k, int j) {
    // 16 elements per thread whatever the batch: the host does not know how
    // many requests are still iterating, and when few are the blocks of the
    // others return at once, so the grid is sized for one request alone
    (void)j;
    return (unsigned)std::max<long long>(1, std::min<long long>(NBLK, cdiv(k.N, (long long)RT * 16)));
}

void launch_arnoldi_dots(const KrylovDev &k, int j, int closing, hipStream_t st) {
    const int G = dots_group(j);
    dim3 grid(dots_blocks(k, j), (unsigned)std::max(1, (int)cdiv(j, G)), k.nb);
#define FM_DOTS(C, GG) hipLaunchKernelGGL((k_arnoldi_dots<C, GG>), grid, dim3(RT), 0, st, k, j)
    if (closing) {
        if (G == 4) FM_DOTS(true, 4);
        else FM_DOTS(true, MD_G);
    } else {
        if (G == 4) FM_DOTS(false, 4);
        else FM_DOTS(false, MD_G);
    }
#undef FM_DOTS
}

void launch_arnoldi_finish(const KrylovDev &k, int j, int closing, hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_finish, dim3(k.nb), dim3(FT), 0, st, k, j, (int)dots_blocks(k, j), closing);
}

void launch_arnoldi_update(const KrylovDev &k, int j, hipStream_t st) {
    if (k.N % 2 == 0) {
        dim3 grid(cdiv(k.N / 2, RT), k.nb);
        hipLaunchKernelGGL(k_arnoldi_update2, grid, dim3(RT), sizeof(double) * (2 * j + 1), st, k, j);
        return;
    }
    dim3 grid(cdiv(k.N, RT), k.nb);
    hipLaunchKernelGGL(k_arnoldi_update, grid, dim3(RT), sizeof(double) * (2 * j + 1), st, k, j);
}

unsigned reduce_blocks(const KrylovDev &k) {
    // every block of a request takes a ticket on one counter when it is done:
    // about 256 blocks over the batch when it is small (1024 serialised
    // tickets cost a single request ~50 us), 32 elements per thread otherwise
    long long nblk = std::max<long long>(cdiv(256, k.nb), cdiv(k.N, (long long)RT * 32));
    return (unsigned)std::max<long long>(1, std::min<long long>(NBLK, nblk));
}

void launch_cycle_solve(const KrylovDev &k, const int *running, hipStream_t st) {
    hipLaunchKernelGGL(k_cycle_solve, dim3(k.nb), dim3(RT), 0, st, k, running);
}

void launch_xupdate(const KrylovDev &k, const int *running, double *x, hipStream_t st) {
    dim3 grid(cdiv(k.N, RT), k.nb);
    hipLaunchKernelGGL(k_xupdate, grid, dim3(RT), 0, st, k, running, x);
}

void launch_residual(const KrylovDev &k, int *running, const double *b, double rtol, double inner_safety,
                     hipStream_t st) {
    dim3 grid(reduce_blocks(k), k.nb);
    hipLaunchKernelGGL(k_residual, grid, dim3(RT), 0, st, k, running, b, rtol, inner_safety);
}

void launch_scale0(const KrylovDev &k, hipStream_t st) {
    dim3 grid(cdiv(k.N, RT), k.nb);
    hipLaunchKernelGGL(k_scale0, grid, dim3(RT), 0, st, k);
}

void launch_bnorm(const KrylovDev &k, const double *b, const int *mask, hipStream_t st) {
    dim3 grid(reduce_blocks(k), k.nb);
    hipLaunchKernelGGL(k_bnorm, grid, dim3(RT), 0, st, k, b, mask);
}

size_t g_lds_limit = 65536;

size_t xy_lds_limit() { return g_lds_limit; }

void prepare_large_lds(size_t bytes) {
    if (bytes > g_lds_limit) g_lds_limit = bytes;
    const void *lp[] = {reinterpret_cast<const void *>(k_xy_lp<1, 1, 4>), reinterpret_cast<const void *>(k_xy_lp<2, 1, 4>),
                        reinterpret_cast<const void *>(k_xy_lp<4, 1, 4>), reinterpret_cast<const void *>(k_xy_lp<4, 1, 8>),
                        reinterpret_cast<const void *>(k_xy_lp<6, 1, 8>), reinterpret_cast<const void *>(k_xy_lp<8, 1, 8>),
                        reinterpret_cast<const void *>(k_xy_lp<1, 2, 4>), reinterpret_cast<const void *>(k_xy_lp<2, 2, 4>),
                        reinterpret_cast<const void *>(k_xy_lp<4, 2, 4>), reinterpret_cast<const void *>(k_xy_lp<4, 2, 8>),
                        reinterpret_cast<const void *>(k_xy_lp<6, 2, 8>), reinterpret_cast<const void *>(k_xy_lp<8, 2, 8>)};
    for (const void *f : lp) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <int QX, int QY, int QZ>
__global__ void __launch_bounds__(256) k_mass_tiled(const ProblemDev *__restrict__ pd, const int *__restrict__ active,
                                                     const double *__restrict__ X, double *__restrict__ Y);

void prepare_operator_lds(size_t bytes) {
    const void *fs[] = {
        reinterpret_cast<const void *>(k_local_grouped<3, 3, 3>), reinterpret_cast<const void *>(k_local_grouped<3, 3, 2>),
        reinterpret_cast<const void *>(k_local_grouped<2, 2, 3>), reinterpret_cast<const void *>(k_local_grouped<2, 2, 2>),
        reinterpret_cast<const void *>(k_local_tiled<3, 3, 3, 2>), reinterpret_cast<const void *>(k_local_tiled<3, 3, 3, 3>),
        reinterpret_cast<const void *>(k_local_tiled<3, 3, 2, 2>), reinterpret_cast<const void *>(k_local_tiled<3, 3, 2, 3>),
        reinterpret_cast<const void *>(k_local_tiled<2, 2, 3, 2>), reinterpret_cast<const void *>(k_local_tiled<2, 2, 3, 3>),
        reinterpret_cast<const void *>(k_local_tiled<2, 2, 2, 2>), reinterpret_cast<const void *>(k_local_tiled<2, 2, 2, 3>),
        reinterpret_cast<const void *>(k_local_many<3, 3, 3>), reinterpret_cast<const void *>(k_local_many<3, 3, 2>),
        reinterpret_cast<const void *>(k_local_many<2, 2, 3>), reinterpret_cast<const void *>(k_local_many<2, 2, 2>),
        reinterpret_cast<const void *>(k_mass_tiled<3, 3, 3>), reinterpret_cast<const void *>(k_mass_tiled<3, 3, 2>),
        reinterpret_cast<const void *>(k_mass_tiled<2, 2, 3>), reinterpret_cast<const void *>(k_mass_tiled<2, 2, 2>)};
    for (const void *f : fs) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

void launch_zero_start(const KrylovDev &k, double *x, const int *mask, int zero_x, hipStream_t st) {
    dim3 grid(cdiv(k.N, 256), k.nb);
    hipLaunchKernelGGL(k_zero_start, grid, dim3(256), 0, st, k, x, mask, zero_x);
}

void launch_fill(double *p, long long n, double v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_copy(double *dst, const double *src, long long n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(cdiv(n, 256)), dim3(256), 0, st, dst, src, n);
}

// ---------------------------------------------------------------------------
// Mass matrix S (Sec. 3.1: the basis products at the collocation points, the
// right-hand matrix of H c = E S c): y = (S_z (x) S_x (x) S_y) x for every
// component and M' block.  One point per thread, all M' blocks; grid
// (points / 256, requests).  For grids that the operator's tiled kernels do
// not cover (k_mass_tiled below for the others).
__global__ void __launch_bounds__(256) k_mass(const ProblemDev *__restrict__ pd, const int *__restrict__ active,
                                              const double *__restrict__ X, double *__restrict__ Y) {
    const int req = blockIdx.y;
    if (active && !active[req]) return;
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int a = 0;
    while (a < 3 && p >= pd->comp[a].npts) {
        p -= pd->comp[a].npts;
        ++a;
    }
    if (a >= 3) return;
    const CompDev &C = pd->comp[a];
    const int nx = C.x.n, ny = C.y.n;
    const int iz = int(p / C.nxy), rem = int(p % C.nxy), ix = rem / ny, iy = rem % ny;
    int gz[MAXR], gx[MAXR], gy[MAXR];
    double Sz[MAXR], Sx[MAXR], Sy[MAXR];
    const int rz = 2 * C.z.q, rx = 2 * C.x.q, ry = 2 * C.y.q;
    for (int t = 0; t < rz; ++t) {
        gz[t] = C.z.idx[iz * MAXR + t];
        Sz[t] = C.z.S[iz * MAXR + t];
    }
    for (int t = 0; t < rx; ++t) {
        gx[t] = C.x.idx[ix * MAXR + t];
        Sx[t] = C.x.S[ix * MAXR + t];
    }
    for (int t = 0; t < ry; ++t) {
        gy[t] = C.y.idx[iy * MAXR + t];
        Sy[t] = C.y.S[iy * MAXR + t];
    }
    for (int iM = 0; iM < pd->nM; ++iM) {
        const long long base = (long long)req * pd->N + C.off + (long long)iM * C.npts;
        const double *c = X + base;
        double sum = 0;
        for (int a1 = 0; a1 < rz; ++a1) {
            if (gz[a1] < 0) continue;
            double bx = 0;
            for (int a2 = 0; a2 < rx; ++a2) {
                if (gx[a2] < 0) continue;
                const double *row = c + ((long long)gz[a1] * nx + gx[a2]) * ny;
                double by = 0;
                for (int a3 = 0; a3 < ry; ++a3)
                    if (gy[a3] >= 0) by += Sy[a3] * row[gy[a3]];
                bx += Sx[a2] * by;
            }
            sum += Sz[a1] * bx;
        }
        Y[base + p] = sum;
    }
}

// The same product on the tiling of the operator's local kernels (a block per
// z point and run of x points, XCD-aware tile order): each M' block's
// coefficients are contracted with the block's z row of S as they are read
// into LDS (one plane over the run's x support x all y), then with each
// point's x and y rows (dropped functions carry the value 0).  active (may be
// null): the rows of the batch to compute.
template <int QX, int QY, int QZ>
__global__ void __launch_bounds__(256) k_mass_tiled(const ProblemDev *__restrict__ pd, const int *__restrict__ active,
                                                     const double *__restrict__ X, double *__restrict__ Y) {
    constexpr int RX = 2 * QX, RY = 2 * QY, RZ = 2 * QZ;
    const int req = blockIdx.y;
    if (active && !active[req]) return;
    extern __shared__ double sm[];
    int t = xcd_tile(blockIdx.x, gridDim.x), a = 0;
    while (a < 3 && t >= pd->comp[a].ntiles) { t -= pd->comp[a].ntiles; ++a; }
    if (a >= 3) return;
    const CompDev &C = pd->comp[a];
    const int ny = C.y.n, xt = C.xt;
    const int ntx = (C.x.n + xt - 1) / xt;
    const int iz = t / ntx, ix0 = (t % ntx) * xt;
    const int nxt = min(xt, C.x.n - ix0);
    const int kxlo = C.x.first[ix0], kxhi = C.x.last[ix0 + nxt - 1];
    const int plane_n = (kxhi - kxlo + 1) * ny;
    const bool has = threadIdx.x < nxt * ny;
    const int ixl = has ? threadIdx.x / ny : 0, iy = has ? threadIdx.x % ny : 0;
    const int ix = ix0 + ixl;
    int lx[RX], ly[RY];
    double Sx[RX], Sy[RY], wz[RZ];
    long long zo[RZ];
#pragma unroll
    for (int q = 0; q < RX; ++q) {
        const int g = C.x.idx[ix * MAXR + q];
        lx[q] = (g >= 0 ? g - kxlo : 0) * ny;
        Sx[q] = C.x.S[ix * MAXR + q];
    }
#pragma unroll
    for (int q = 0; q < RY; ++q) {
        const int g = C.y.idx[iy * MAXR + q];
        ly[q] = g >= 0 ? g : 0;
        Sy[q] = C.y.S[iy * MAXR + q];
    }
#pragma unroll
    for (int q = 0; q < RZ; ++q) {
        const int g = C.z.idx[iz * MAXR + q];
        zo[q] = (long long)(g >= 0 ? g : 0) * C.nxy;
        wz[q] = C.z.S[iz * MAXR + q];
    }
    const long long p = (long long)iz * C.nxy + ix * ny + iy;
    const double *xr = X + (long long)req * pd->N + C.off + (long long)kxlo * ny;
    double *yr = Y + (long long)req * pd->N + C.off + p;
    const int nM = pd->nM;
    for (int iM = 0; iM < nM; ++iM) {
        __syncthreads();                     // the previous block's plane is read
        const double *xb = xr + (long long)iM * C.npts;
        for (int e = threadIdx.x; e < plane_n; e += 256) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < RZ; ++q) v += wz[q] * xb[zo[q] + e];
            sm[e] = v;
        }
        __syncthreads();
        if (has) {
            double sum = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < RX; ++q2) {
                double ty = 0.0;
#pragma unroll
                for (int q3 = 0; q3 < RY; ++q3) ty += Sy[q3] * sm[lx[q2] + ly[q3]];
                sum += Sx[q2] * ty;
            }
            yr[(long long)iM * C.npts] = sum;
        }
    }
}

void launch_mass(const ProblemDev &pd, int nb, const double *x, double *y, hipStream_t st, const int *active) {
    if (matvec_tiled_ok(pd)) {
        const unsigned tiles = (pd.comp[0].ntiles + pd.comp[1].ntiles + pd.comp[2].ntiles + 7) & ~7u;
        const size_t lds = sizeof(double) * size_t(pd.plane_lds / 3 + 1);
        dim3 grid(tiles, nb);
        switch ((pd.q[0] == 3 ? 2 : 0) + (pd.q[2] == 3 ? 1 : 0)) {
            case 3: hipLaunchKernelGGL((k_mass_tiled<3, 3, 3>), grid, dim3(256), lds, st, pd.dev, active, x, y); return;
            case 2: hipLaunchKernelGGL((k_mass_tiled<3, 3, 2>), grid, dim3(256), lds, st, pd.dev, active, x, y); return;
            case 1: hipLaunchKernelGGL((k_mass_tiled<2, 2, 3>), grid, dim3(256), lds, st, pd.dev, active, x, y); return;
            default: hipLaunchKernelGGL((k_mass_tiled<2, 2, 2>), grid, dim3(256), lds, st, pd.dev, active, x, y); return;
        }
    }
    long long pts = 0;
    for (int a = 0; a < 3; ++a) pts += pd.comp[a].npts;
    dim3 grid(cdiv(pts, 256), nb);
    hipLaunchKernelGGL(k_mass, grid, dim3(256), 0, st, pd.dev, active, x, y);
}

// ---------------------------------------------------------------------------
// Column kernels of the eigenvalue iteration.  A basis of ncol columns of
// length N is stored column after column (column c at V + c * N).

// part[c * nblk + b] = (this block's share of) V_c . w; grid (nblk, ncol).
__global__ void __launch_bounds__(256) k_cols_dot_part(const double *__restrict__ V, const double *__restrict__ w,
                                                       long long N, double *__restrict__ part, int nblk) {
    const int c = blockIdx.y;
    const double *v = V + (long long)c * N;
    double s = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < N; i += (long long)nblk * 256) s += v[i] * w[i];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)c * nblk + blockIdx.x] = red[0];
}

// out[c] = sum of the nblk partials of column c in block order; grid (ncol).
__global__ void __launch_bounds__(256) k_cols_dot_finish(const double *__restrict__ part, int nblk,
                                                         double *__restrict__ out) {
    const int c = blockIdx.x;
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[(long long)c * nblk + b];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// w -= sum_c V_c h[c]
__global__ void __launch_bounds__(256) k_cols_axpy(double *__restrict__ w, const double *__restrict__ V, int ncol,
                                                   const double *__restrict__ h, long long N) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    double s = w[i];
    for (int c = 0; c < ncol; ++c) s -= V[(long long)c * N + i] * h[c];
    w[i] = s;
}

// out_c = sum_j V_j Y[j * k + c] for c < k (Y row-major m x k); grid (N / 256, k)
__global__ void __launch_bounds__(256) k_cols_combine(const double *__restrict__ V, int m, const double *__restrict__ Y,
                                                      int k, double *__restrict__ out, long long N) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= N) return;
    double s = 0;
    for (int j = 0; j < m; ++j) s += V[(long long)j * N + i] * Y[j * k + c];
    out[(long long)c * N + i] = s;
}

__global__ void __launch_bounds__(256) k_scale_vec(double *__restrict__ w, double s, long long N) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < N) w[i] *= s;
}

int cols_dot_blocks(long long N) { return (int)std::max<long long>(1, std::min<long long>(NBLK, cdiv(N, 256 * 8))); }

void launch_cols_dot(const double *V, int ncol, const double *w, long long N, double *part, double *out,
                     hipStream_t st) {
    const int nblk = cols_dot_blocks(N);
    hipLaunchKernelGGL(k_cols_dot_part, dim3(nblk, ncol), dim3(256), 0, st, V, w, N, part, nblk);
    hipLaunchKernelGGL(k_cols_dot_finish, dim3(ncol), dim3(256), 0, st, part, nblk, out);
}

void launch_cols_axpy(double *w, const double *V, int ncol, const double *h, long long N, hipStream_t st) {
    hipLaunchKernelGGL(k_cols_axpy, dim3(cdiv(N, 256)), dim3(256), 0, st, w, V, ncol, h, N);
}

void launch_cols_combine(const double *V, int m, const double *Y, int k, double *out, long long N, hipStream_t st) {
    hipLaunchKernelGGL(k_cols_combine, dim3(cdiv(N, 256), k), dim3(256), 0, st, V, m, Y, k, out, N);
}

void launch_scale_vec(double *w, double s, long long N, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_vec, dim3(cdiv(N, 256)), dim3(256), 0, st, w, s, N);
}


// ---------------------------------------------------------------------------
// Complex energies.  A complex request is a pair of real rows (real part,
// imaginary part) of one problem, [request][re, im][N]; the operator and the
// preconditioner's transforms are real, so they act on the two rows as two
// requests, and only the divide and the E S term couple the rows.

struct cplx {
    double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cscale(double s, cplx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cplx cquot(cplx a, cplx b) {
    const double q = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / q, (a.im * b.re - a.re * b.im) / q};
}
__device__ __forceinline__ double cabs2(cplx a) { return sqrt(a.re * a.re + a.im * a.im); }

// (Lambda_x (x) I + I (x) Lambda_y - E)^-1 on one slice of every complex
// request, in place, with E complex (Sec. 3.2, eq. (prec-2)): the closed forms
// of the real divide (one complex division per real pair of eigenvalues; the
// 2x2 and 4x4 blocks of complex-conjugate eigenpairs) hold with the shifted
// diagonal d = lambda_x + lambda_y - E complex, and the data of each element
// is complex (its two rows).  One thread per anchor element of a block; grid
// (slices, element chunks of 256, complex requests).  min_den[c]: minimum
// modulus over the blocks' eigenvalues of lambda - E.
__global__ void __launch_bounds__(256) k_cdivide(const ProblemDev *__restrict__ pd, const PrecDev *__restrict__ pr,
                                                 const double *__restrict__ Ere, const double *__restrict__ Eim,
                                                 const int *__restrict__ active, double *data, double *min_den) {
    const int c = blockIdx.z;
    if (active && !active[c]) return;
    int a, iM, k;
    if (!slice_decode(pd, blockIdx.x, a, iM, k)) return;
    const CompDev &C = pd->comp[a];
    const PrecCompDev &F = pr->comp[a];
    const int nx = C.x.n, ny = C.y.n, nz = C.z.n;
    const size_t fx = (size_t)iM * nz + k;
    const double *lx = F.lx + fx * nx, *lxi = F.lxi + fx * nx, *ly = F.ly + fx * ny, *lyi = F.lyi + fx * ny;
    const signed char *tx = F.tx + fx * nx, *ty = F.ty + fx * ny;
    const long long off = C.off + (long long)iM * C.npts + (long long)k * C.nxy;
    double *re = data + (long long)(2 * c) * pd->N + off, *im = data + (long long)(2 * c + 1) * pd->N + off;
    const cplx E = {Ere[c], Eim[c]};
    double mind = 1e300;
    const int e = blockIdx.y * 256 + threadIdx.x;
    if (e < nx * ny) {
        const int i = e / ny, j = e % ny, o = i * ny + j;
        const int ti = tx[i], tj = ty[j];
        if (ti != 2 && tj != 2) {
            const cplx d = csub({lx[i] + ly[j], 0.0}, E);
            if (ti == 0 && tj == 0) {
                const cplx t = cquot({re[o], im[o]}, d);
                re[o] = t.re;
                im[o] = t.im;
                mind = cabs2(d);
            } else if (tj == 0 || ti == 0) {
                // one complex pair (rows i, i + 1 or columns j, j + 1): the block
                // [[d, b], [-b, d]] inverted; eigenvalues d +- i b
                const double b = tj == 0 ? lxi[i] : lyi[j];
                const int o1 = tj == 0 ? o + ny : o + 1;
                const cplx r0 = {re[o], im[o]}, r1 = {re[o1], im[o1]};
                const cplx det = cadd(cmul(d, d), {b * b, 0.0});
                const cplx t0 = cquot(csub(cmul(d, r0), cscale(b, r1)), det);
                const cplx t1 = cquot(cadd(cscale(b, r0), cmul(d, r1)), det);
                re[o] = t0.re;
                im[o] = t0.im;
                re[o1] = t1.re;
                im[o1] = t1.im;
                mind = fmin(cabs2(cadd(d, {0.0, b})), cabs2(csub(d, {0.0, b})));
            } else {
                // both in pairs: split on the eigenspaces of the two commuting
                // structures into divisions by d +- i (bx - by), d +- i (bx + by)
                const double bx = lxi[i], by = lyi[j];
                const cplx r00 = {re[o], im[o]}, r01 = {re[o + 1], im[o + 1]};
                const cplx r10 = {re[o + ny], im[o + ny]}, r11 = {re[o + ny + 1], im[o + ny + 1]};
                const cplx p00 = cscale(0.5, cadd(r00, r11)), p01 = cscale(0.5, csub(r01, r10));
                const cplx m00 = cscale(0.5, csub(r00, r11)), m01 = cscale(0.5, cadd(r01, r10));
                const double bp = bx - by, bm = bx + by;
                const cplx Dp = cadd(cmul(d, d), {bp * bp, 0.0}), Dm = cadd(cmul(d, d), {bm * bm, 0.0});
                const cplx t00 = cadd(cquot(cadd(cmul(d, p00), cscale(bp, p01)), Dp),
                                      cquot(csub(cmul(d, m00), cscale(bm, m01)), Dm));
                const cplx t01 = cadd(cquot(csub(cmul(d, p01), cscale(bp, p00)), Dp),
                                      cquot(cadd(cmul(d, m01), cscale(bm, m00)), Dm));
                const cplx t10 = cadd(cquot(cadd(cscale(-1.0, cmul(d, p01)), cscale(bp, p00)), Dp),
                                      cquot(cadd(cmul(d, m01), cscale(bm, m00)), Dm));
                const cplx t11 = cadd(cquot(cadd(cmul(d, p00), cscale(bp, p01)), Dp),
                                      cquot(cadd(cscale(-1.0, cmul(d, m00)), cscale(bm, m01)), Dm));
                re[o] = t00.re;
                im[o] = t00.im;
                re[o + 1] = t01.re;
                im[o + 1] = t01.im;
                re[o + ny] = t10.re;
                im[o + ny] = t10.im;
                re[o + ny + 1] = t11.re;
                im[o + ny + 1] = t11.im;
                mind = fmin(fmin(cabs2(cadd(d, {0.0, bp})), cabs2(csub(d, {0.0, bp}))),
                            fmin(cabs2(cadd(d, {0.0, bm})), cabs2(csub(d, {0.0, bm}))));
            }
        }
    }
    if (min_den) block_min_store(mind, min_den + c);
}

// y_re += E_im (S x)_im, y_im -= E_im (S x)_re for every complex request:
// the imaginary part of the energy term of (H - E S) x once A(Re E) has been
// applied to both rows.  sx: S x of both rows.  Grid (chunks of N, requests).
__global__ void __launch_bounds__(256) k_cplx_energy(double *__restrict__ y, const double *__restrict__ sx,
                                                     const double *__restrict__ Eim, const int *__restrict__ active,
                                                     long long N) {
    const int c = blockIdx.y;
    if (active && !active[c]) return;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double e = Eim[c];
    double *yr = y + (long long)(2 * c) * N, *yi = yr + N;
    const double *sr = sx + (long long)(2 * c) * N, *si = sr + N;
    const double a = sr[i], b = si[i];
    yr[i] += e * b;
    yi[i] -= e * a;
}

// out[2c] = out[2c + 1] = in[c]: a per-request mask for the rows of complex requests.
__global__ void k_expand_mask(const int *__restrict__ in, int *__restrict__ out, int n) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < n) {
        const int v = in[c];
        out[2 * c] = v;
        out[2 * c + 1] = v;
    }
}

void launch_cdivide(const ProblemDev &pd, const PrecDev &pr, int nbc, const double *Ere, const double *Eim,
                    const int *active, double *data, double *min_den, hipStream_t st) {
    int slices = 0, maxnxy = 0;
    for (int a = 0; a < 3; ++a) {
        slices += pd.nM * pd.comp[a].z.n;
        maxnxy = std::max(maxnxy, pd.comp[a].nxy);
    }
    hipLaunchKernelGGL(k_cdivide, dim3(slices, cdiv(maxnxy, 256), nbc), dim3(256), 0, st, pd.dev, pr.dev, Ere, Eim,
                       active, data, min_den);
}

void launch_cplx_energy(double *y, const double *sx, const double *Eim, const int *active, int nbc, long long N,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_cplx_energy, dim3(cdiv(N, 256), nbc), dim3(256), 0, st, y, sx, Eim, active, N);
}

void launch_expand_mask(const int *in, int *out, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_expand_mask, dim3(cdiv(n, 256)), dim3(256), 0, st, in, out, n);
}

// Two of the four staged x-y products over every slice of nrows rows, in
// place through tmp: which 0, data <- Wbar_x data Wbar_y^T; which 1,
// data <- W_x data W_y^T (no divide: the complex path divides in between).
void launch_xy_half(const ProblemDev &pd, const PrecDev &pr, int nrows, const int *active, int which, double *data,
                    double *tmp, hipStream_t st) {
    int slices = 0, side = 0;
    long long t64 = 0, area64 = 0, area32 = 0;
    for (int a = 0; a < 3; ++a) {
        slices += pd.nM * pd.comp[a].z.n;
        const int nx = pd.comp[a].x.n, ny = pd.comp[a].y.n;
        side = std::max(side, std::max(nx, ny));
        t64 = std::max<long long>(t64, (long long)sg_tiles(nx, 64) * sg_tiles(ny, 64));
        area64 += 4096LL * sg_tiles(nx, 64) * sg_tiles(ny, 64);
        area32 += 1024LL * sg_tiles(nx, 32) * sg_tiles(ny, 32);
    }
#define FM_XYH(BT)                                                                                                   \
    {                                                                                                                \
        int tl = 0;                                                                                                  \
        for (int a = 0; a < 3; ++a) tl = std::max(tl, sg_tiles(pd.comp[a].x.n, BT) * sg_tiles(pd.comp[a].y.n, BT)); \
        const dim3 g(slices, tl, nrows);                                                                             \
        hipLaunchKernelGGL((k_slice_gemm<true, false, false, BT>), g, dim3(256), 0, st, pd.dev, pr.dev, nullptr,     \
                           active, which, data, tmp, nullptr);                                                       \
        hipLaunchKernelGGL((k_slice_gemm<false, false, false, BT>), g, dim3(256), 0, st, pd.dev, pr.dev, nullptr,    \
                           active, which, tmp, data, nullptr);                                                       \
    }
    if (side > 32 && t64 * slices * nrows >= XY_T64_MIN_BLOCKS && 4 * area64 <= 5 * area32) FM_XYH(64) else FM_XYH(32)
#undef FM_XYH
}

}  // namespace fm
