// Fluid model on the octree: one explicit stage of the drift-diffusion-
// reaction equations for the electron and ion densities (paper section 2.2;
// fluxes, limiter, refinement-boundary treatment and the coefficient table:
// section 2.3; the trapezoidal stages and the time-step limits: section 2.4),
//   out_e = wa n0_e + wb (n_e + dt (S - div F)),  out_i = wa n0_i + wb (n_i + dt S),
// with S = alpha(E) mu(E) E n_e at the cell centre (E = |E|) and F the
// electron flux across each face: v n_face - D(E*) (n_R - n_L) / h, where
// v = -mu(E*) E_a, E_a the face component of the field, E* the mean |E| of the
// two cells and n_face the upwind value corrected with the Koren limiter.
//
// Densities are natural-layout [box][k][j][i] arrays.  Outside a box they
// come from the same-level box (its covered cells hold the mean of their
// children: k_fluid_restrict), from the mirrored interior cell at the domain
// boundary (zero gradient), or, across a refinement boundary, from a fine
// ghost = 1/4 of the coarse cell holding it + 1/4 of that cell's three
// neighbours on the ghost's side (linear interpolation), capped at twice the
// coarse value.  The faces of a refinement boundary are computed once, from
// the fine side, per slot (k_fluid_cf); the coarse box takes the mean of the
// four fine fluxes on each of its face cells, so no mass is lost there.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mg {

namespace {

constexpr double kCharge = 1.602176634e-19;  // elementary charge, C
constexpr double kEps0 = 8.8541878128e-12;   // vacuum permittivity, F/m

__device__ __forceinline__ void axes(int a, int &t1, int &t2) {
    t1 = a == 0 ? 1 : 0;
    t2 = a == 2 ? 1 : 2;
}
__device__ __forceinline__ int nat(const int c[3]) { return (c[2] * 8 + c[1]) * 8 + c[0]; }
// cell (x, y, z) at position pa along axis a and (u, v) along its tangential
// axes (t1, t2)
struct Cell {
    int x, y, z;
};
__device__ __forceinline__ Cell place(int a, int pa, int u, int v) {
    Cell c;
    c.x = a == 0 ? pa : u;
    c.y = a == 0 ? u : (a == 1 ? pa : v);
    c.z = a == 2 ? pa : v;
    return c;
}
__device__ __forceinline__ int natc(Cell c) { return (c.z * 8 + c.y) * 8 + c.x; }
// colour-split position of cell (i, j, k) in the solver's fields
__device__ __forceinline__ int cs_pos(int i, int j, int k) {
    return (((i + j + k) & 1) << 8) + ((k * 8 + j) << 2) + (i >> 1);
}
__device__ __forceinline__ int64_t xcd_pos(int64_t blk, int64_t n) {
    int64_t per = (n + 7) >> 3;
    return (blk & 7) * per + (blk >> 3);
}

// Position of field strength E in the table: interval row k and weight w
// (linear interpolation between entries k and k+1; beyond emax the last
// row, which repeats entry n-1, with w = 0)
__device__ __forceinline__ const double2 *tab_row(const FluidTable &T, double E, double &w) {
    double x = E * T.scale;
    int k = (int)floor(x);
    if (k >= T.n - 1 || !(x >= 0.0)) {
        k = k >= T.n - 1 ? T.n - 1 : 0;
        w = 0.0;
    } else {
        w = x - (double)k;
    }
    return reinterpret_cast<const double2 *>(T.v + 6 * (int64_t)k);
}
__device__ __forceinline__ double lerp(double2 p, double w) { return (1.0 - w) * p.x + w * p.y; }
// mu and D at E (two 16-byte loads)
__device__ __forceinline__ void coef2(const FluidTable &T, double E, double &mu, double &D) {
    double w;
    const double2 *r = tab_row(T, E, w);
    mu = lerp(r[0], w);
    D = lerp(r[1], w);
}
// mu, D and alpha at E (three 16-byte loads)
__device__ __forceinline__ void coef(const FluidTable &T, double E, double &mu, double &D, double &al) {
    double w;
    const double2 *r = tab_row(T, E, w);
    mu = lerp(r[0], w);
    D = lerp(r[1], w);
    al = lerp(r[2], w);
}

// Minimum that carries NaN through (fmin drops it): the time-step bound of a
// stage with a non-finite output is NaN.
__device__ __forceinline__ double nanmin(double a, double b) {
    return (a != a || a < b) ? a : b;
}

// psi(a / b) * b for the Koren limiter psi(x) = max(0, min(1, (2 + x) / 6, x)),
// without the division: for b > 0 it is max(0, min(b, (2b + a) / 6, a)), for
// b < 0 the same with min and max exchanged, and 0 for b = 0
__device__ __forceinline__ double koren(double a, double b) {
    const double sixth = 1.0 / 6.0;
    if (b > 0.0) return fmax(0.0, fmin(b, fmin((2.0 * b + a) * sixth, a)));
    if (b < 0.0) return fmin(0.0, fmax(b, fmax((2.0 * b + a) * sixth, a)));
    return 0.0;
}

// flux across the face between cells L = f-1 and R = f, from the densities
// of cells f-2, f-1, f, f+1
__device__ __forceinline__ double flux(double m2, double m1, double p0, double p1, double vel, double D,
                                       double inv_h) {
    double b = p0 - m1;
    double nf = vel < 0.0 ? p0 - koren(p1 - p0, b) : m1 + koren(m1 - m2, b);
    return vel * nf - D * b * inv_h;
}

__device__ __forceinline__ double cell_h(const Geo &g, int l) { return g.len / (8.0 * (double)(1 << (l - 1))); }

// covered cells of the parent of every leaf box (level >= 2) <- mean of the
// box's 8 cells under each; 64 threads per leaf box
__global__ __launch_bounds__(64) void k_fluid_restrict(Geo g, double *__restrict__ n,
                                                       const int32_t *__restrict__ leaf, int64_t nleaf) {
    int64_t q = blockIdx.x;
    if (q >= nleaf) return;
    int64_t b = leaf[q];
    if (g.ijk[b * 4 + 3] < 2) return;
    int64_t p = g.parent[b];
    int t = threadIdx.x, pi = t & 3, pj = (t >> 2) & 3, pk = t >> 4;
    const double *f = n + b * 512;
    double s = 0.0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int di = 0; di < 2; di++) s += f[((2 * pk + dk) * 8 + 2 * pj + dj) * 8 + 2 * pi + di];
    int c[3] = {4 * (g.ijk[b * 4] & 1) + pi, 4 * (g.ijk[b * 4 + 1] & 1) + pj, 4 * (g.ijk[b * 4 + 2] & 1) + pk};
    n[p * 512 + nat(c)] = 0.125 * s;
}

// One refinement-boundary face per workgroup (slot s: fine box B, face d),
// one face cell (u, v) per thread: the two fine ghosts across the face, the
// flux on it and the face velocity -> cf[s][0..3][64].
__global__ __launch_bounds__(64) void k_fluid_cf(Geo g, const double *__restrict__ n,
                                                 const double *__restrict__ ef, const double *__restrict__ en,
                                                 FluidTable T, const int32_t *__restrict__ slots,
                                                 int64_t nslot, double *__restrict__ cf) {
    int64_t s = blockIdx.x;
    if (s >= nslot) return;
    int64_t B = slots[2 * s];
    int d = slots[2 * s + 1], a = d >> 1, side = d & 1, t1, t2;
    axes(a, t1, t2);
    int q = threadIdx.x, u = q & 7, v = q >> 3;
    const int32_t *x = g.slotx + 8 * s;  // Q, base t1, base t2, Q's neighbours -t1 +t1 -t2 +t2
    int64_t Q = x[0];
    int64_t P = g.parent[B];
    double inv_h = 1.0 / cell_h(g, g.ijk[B * 4 + 3]);
    int C[3];
    C[a] = side ? 0 : 7;
    C[t1] = x[1] + (u >> 1);
    C[t2] = x[2] + (v >> 1);
    double cc = n[Q * 512 + nat(C)];
    double gh[2];
#pragma unroll
    for (int L = 0; L < 2; L++) {
        double nbv[3];
        // normal: the adjacent ghost's neighbour lies toward B (a covered cell
        // of B's parent), the outer ghost's inside Q
        {
            bool toward = L == 0;
            int D[3] = {C[0], C[1], C[2]};
            if (toward) {
                D[a] = side ? 7 : 0;
                nbv[a] = n[P * 512 + nat(D)];
            } else {
                D[a] = side ? 1 : 6;
                nbv[a] = n[Q * 512 + nat(D)];
            }
        }
        // tangential: the side of the fine cell within the coarse cell
#pragma unroll
        for (int w = 0; w < 2; w++) {
            int ax = w ? t2 : t1, par = w ? (v & 1) : (u & 1);
            int D[3] = {C[0], C[1], C[2]};
            D[ax] += par ? 1 : -1;
            double val;
            if (D[ax] >= 0 && D[ax] < 8) {
                val = n[Q * 512 + nat(D)];
            } else {
                int N = x[3 + 2 * w + (par ? 1 : 0)];
                if (N >= 0) {
                    D[ax] = par ? 0 : 7;
                    val = n[(int64_t)N * 512 + nat(D)];
                } else {
                    val = cc;  // domain boundary: the mirrored cell is C itself
                }
            }
            nbv[ax] = val;
        }
        double gv = 0.25 * cc + 0.25 * (nbv[0] + nbv[1] + nbv[2]);
        gh[L] = gv < 2.0 * cc ? gv : 2.0 * cc;
    }
    double eg = en[Q * 512 + nat(C)];
    int c[3];
    c[t1] = u;
    c[t2] = v;
    double m2, m1, p0, p1, eL, eR;
    int f;
    if (side == 0) {  // face 0 of B: ghosts at -2, -1
        f = 0;
        c[a] = 0;
        p0 = n[B * 512 + nat(c)];
        eR = en[B * 512 + nat(c)];
        c[a] = 1;
        p1 = n[B * 512 + nat(c)];
        m2 = gh[1];
        m1 = gh[0];
        eL = eg;
    } else {  // face 8: ghosts at 8, 9
        f = 8;
        c[a] = 6;
        m2 = n[B * 512 + nat(c)];
        c[a] = 7;
        m1 = n[B * 512 + nat(c)];
        eL = en[B * 512 + nat(c)];
        p0 = gh[0];
        p1 = gh[1];
        eR = eg;
    }
    double mu, D;
    coef2(T, 0.5 * (eL + eR), mu, D);
    double vel = -mu * ef[((B * 3 + a) * 9 + f) * 64 + q];
    double* o = cf + s * 256;
    o[q] = gh[0];
    o[64 + q] = gh[1];
    o[128 + q] = flux(m2, m1, p0, p1, vel, D, inv_h);
    o[192 + q] = vel;
}

// One leaf box per workgroup, one cell per thread: the densities with two
// ghost layers and |E| with one in LDS, every face flux and velocity of the
// box, then the update of the cell, the solver's right-hand side
// -e (n_i - n_e) / eps0 and the box's time-step bound.
__global__ __launch_bounds__(512) void k_fluid_update(
    Geo g, const int32_t *__restrict__ isleaf, const int32_t *__restrict__ cfrev,
    const int32_t *__restrict__ leaf, int64_t nleaf, const double *__restrict__ ne,
    const double *__restrict__ ni, const double *__restrict__ n0e, const double *__restrict__ n0i,
    const double *__restrict__ ef, const double *__restrict__ en, FluidTable T,
    const double *__restrict__ cf, double dt, double wa, double wb, double *__restrict__ oute,
    double *__restrict__ outi, double *__restrict__ rhs, double *__restrict__ partial) {
    __shared__ double N[12 * 12 * 12], EN[10 * 10 * 10], FX[1728], VX[1728], red[8];
    int64_t q = xcd_pos(blockIdx.x, nleaf);
    if (q >= nleaf) return;
    int64_t b = leaf[q];
    int t = threadIdx.x, i = t & 7, j = (t >> 3) & 7, k = t >> 6;
    auto p2 = [](int x, int y, int z) { return ((z + 2) * 12 + (y + 2)) * 12 + (x + 2); };
    auto p1 = [](int x, int y, int z) { return ((z + 1) * 10 + (y + 1)) * 10 + (x + 1); };
    int nb[6], sl[6];
#pragma unroll
    for (int d = 0; d < 6; d++) {
        nb[d] = g.nbr[b * 6 + d];
        sl[d] = g.cfslot[b * 6 + d];
    }
    double h = cell_h(g, g.ijk[b * 4 + 3]), inv_h = 1.0 / h;
    double nec = ne[b * 512 + t], nic = ni[b * 512 + t], n0ec = n0e[b * 512 + t], n0ic = n0i[b * 512 + t];
    double enc = en[b * 512 + t];
    N[p2(i, j, k)] = nec;
    EN[p1(i, j, k)] = enc;
    // density ghosts: face d, layer L (0 adjacent), face cell (u, v)
    for (int e = t; e < 768; e += 512) {
        int d = e >> 7, L = (e >> 6) & 1, qq = e & 63, a = d >> 1, side = d & 1;
        int u = qq & 7, v = qq >> 3;
        int nbd = d == 0 ? nb[0] : d == 1 ? nb[1] : d == 2 ? nb[2] : d == 3 ? nb[3] : d == 4 ? nb[4] : nb[5];
        int sld = d == 0 ? sl[0] : d == 1 ? sl[1] : d == 2 ? sl[2] : d == 3 ? sl[3] : d == 4 ? sl[4] : sl[5];
        double val;
        if (nbd >= 0) {
            val = ne[(int64_t)nbd * 512 + natc(place(a, side ? L : 7 - L, u, v))];
        } else if (nbd == -2) {
            val = ne[b * 512 + natc(place(a, side ? 7 - L : L, u, v))];
        } else {
            val = cf[(int64_t)sld * 256 + L * 64 + qq];
        }
        Cell c = place(a, side ? 8 + L : -1 - L, u, v);
        N[p2(c.x, c.y, c.z)] = val;
    }
    // |E| ghosts (one layer): the same-level cell, the mirrored cell, or the
    // coarse cell holding the ghost
    if (t < 384) {
        int d = t >> 6, qq = t & 63, a = d >> 1, side = d & 1;
        int u = qq & 7, v = qq >> 3;
        int nbd = d == 0 ? nb[0] : d == 1 ? nb[1] : d == 2 ? nb[2] : d == 3 ? nb[3] : d == 4 ? nb[4] : nb[5];
        int sld = d == 0 ? sl[0] : d == 1 ? sl[1] : d == 2 ? sl[2] : d == 3 ? sl[3] : d == 4 ? sl[4] : sl[5];
        double val;
        if (nbd >= 0) {
            val = en[(int64_t)nbd * 512 + natc(place(a, side ? 0 : 7, u, v))];
        } else if (nbd == -2) {
            val = en[b * 512 + natc(place(a, side ? 7 : 0, u, v))];
        } else {
            const int32_t *x = g.slotx + 8 * (int64_t)sld;
            val = en[(int64_t)x[0] * 512 + natc(place(a, side ? 0 : 7, x[1] + (u >> 1), x[2] + (v >> 1)))];
        }
        Cell c = place(a, side ? 8 : -1, u, v);
        EN[p1(c.x, c.y, c.z)] = val;
    }
    __syncthreads();
    // faces: axis a, face f = 0..8 (between cells f-1 and f), cell (u, v)
    for (int e = t; e < 1728; e += 512) {
        int a = e / 576, r = e - 576 * a, f = r >> 6, qq = r & 63;
        int u = qq & 7, v = qq >> 3;
        Cell cl = place(a, f - 1, u, v), cr = place(a, f, u, v);
        double eL = EN[p1(cl.x, cl.y, cl.z)], eR = EN[p1(cr.x, cr.y, cr.z)];
        double mu, D;
        coef2(T, 0.5 * (eL + eR), mu, D);
        double V = -mu * ef[((b * 3 + a) * 9 + f) * 64 + qq], F;
        int d = 2 * a + (f == 8 ? 1 : 0);
        int nbd = d == 0 ? nb[0] : d == 1 ? nb[1] : d == 2 ? nb[2] : d == 3 ? nb[3] : d == 4 ? nb[4] : nb[5];
        int sld = d == 0 ? sl[0] : d == 1 ? sl[1] : d == 2 ? sl[2] : d == 3 ? sl[3] : d == 4 ? sl[4] : sl[5];
        bool bnd = f == 0 || f == 8;
        if (bnd && nbd == -1) {  // fine side of a refinement boundary
            F = cf[(int64_t)sld * 256 + 128 + qq];
            V = cf[(int64_t)sld * 256 + 192 + qq];
        } else if (bnd && nbd >= 0 && !isleaf[nbd]) {  // coarse side: mean of the 4 fine fluxes
            int64_t fs = cfrev[(b * 6 + d) * 4 + (v >> 2) * 2 + (u >> 2)];
            double s = 0.0;
            for (int dv = 0; dv < 2; dv++)
                for (int du = 0; du < 2; du++)
                    s += cf[fs * 256 + 128 + ((2 * v + dv) & 7) * 8 + ((2 * u + du) & 7)];
            F = 0.25 * s;
        } else {
            Cell c0 = place(a, f - 2, u, v), c3 = place(a, f + 1, u, v);
            F = flux(N[p2(c0.x, c0.y, c0.z)], N[p2(cl.x, cl.y, cl.z)], N[p2(cr.x, cr.y, cr.z)],
                     N[p2(c3.x, c3.y, c3.z)], V, D, inv_h);
        }
        FX[e] = F;
        VX[e] = V;
    }
    __syncthreads();
    double div = 0.0, vs = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        // the cell's faces along a: position f0, tangential (t1, t2) cell qa
        int f0 = a == 0 ? i : (a == 1 ? j : k);
        int qa = a == 0 ? k * 8 + j : (a == 1 ? k * 8 + i : j * 8 + i);
        div += (FX[a * 576 + (f0 + 1) * 64 + qa] - FX[a * 576 + f0 * 64 + qa]) * inv_h;
        double v0 = fabs(VX[a * 576 + f0 * 64 + qa]), v1 = fabs(VX[a * 576 + (f0 + 1) * 64 + qa]);
        vs += (v0 > v1 ? v0 : v1) * inv_h;
    }
    double mu, D, al;
    coef(T, enc, mu, D, al);
    double S = al * mu * enc * nec;
    double oe = wa * n0ec + wb * (nec + dt * (S - div));
    double oi = wa * n0ic + wb * (nic + dt * S);
    oute[b * 512 + t] = oe;
    outi[b * 512 + t] = oi;
    rhs[b * 512 + cs_pos(i, j, k)] = -kCharge * (oi - oe) / kEps0;
    // time-step bound of the cell: CFL 0.5, advection + diffusion 1,
    // dielectric relaxation
    double cand = INFINITY;
    if (vs > 0.0) cand = 0.5 / vs;
    double ad = 1.0 / (vs + 6.0 * D / (h * h));
    if (ad < cand) cand = ad;
    if (nec > 0.0 && mu > 0.0) {
        double dr = kEps0 / (kCharge * mu * nec);
        if (dr < cand) cand = dr;
    }
    // a non-finite output poisons the bound, so a diverging step is seen
    if (!isfinite(oe) || !isfinite(oi)) cand = NAN;
    for (int off = 32; off > 0; off >>= 1) cand = nanmin(cand, __shfl_xor(cand, off));
    if ((t & 63) == 0) red[t >> 6] = cand;
    __syncthreads();
    if (t == 0) {
        double m = red[0];
        for (int w = 1; w < 8; w++) m = nanmin(m, red[w]);
        partial[q] = m;
    }
}

// out[0] = min over partial[0..n)
__global__ __launch_bounds__(1024) void k_fluid_min(const double *__restrict__ partial, int64_t n,
                                                    double *__restrict__ out) {
    __shared__ double red[16];
    int t = threadIdx.x;
    double m = INFINITY;
    for (int64_t q = t; q < n; q += 1024) m = nanmin(m, partial[q]);
    for (int off = 32; off > 0; off >>= 1) m = nanmin(m, __shfl_xor(m, off));
    if ((t & 63) == 0) red[t >> 6] = m;
    __syncthreads();
    if (t == 0) {
        double r = red[0];
        for (int w = 1; w < 16; w++) r = nanmin(r, red[w]);
        out[0] = r;
    }
}

}  // namespace

void launch_fluid_stage(const Geo &g, const FluidArgs &A, hipStream_t s) {
    if (A.nleaf > 0)
        hipLaunchKernelGGL(k_fluid_restrict, dim3((unsigned)A.nleaf), dim3(64), 0, s, g, A.ne, A.leaf,
                           A.nleaf);
    if (A.nslot > 0)
        hipLaunchKernelGGL(k_fluid_cf, dim3((unsigned)A.nslot), dim3(64), 0, s, g, (const double *)A.ne, A.ef,
                           A.en, A.tab, A.slots, A.nslot, A.cf);
    if (A.nleaf > 0) {
        hipLaunchKernelGGL(k_fluid_update, dim3((unsigned)(8 * ((A.nleaf + 7) >> 3))), dim3(512), 0, s, g,
                           A.isleaf, A.cfrev, A.leaf, A.nleaf, (const double *)A.ne, A.ni, A.n0e, A.n0i,
                           A.ef, A.en, A.tab, (const double *)A.cf, A.dt, A.wa, A.wb, A.oute, A.outi,
                           A.rhs, A.partial);
        hipLaunchKernelGGL(k_fluid_min, dim3(1), dim3(1024), 0, s, (const double *)A.partial, A.nleaf,
                           A.result);
    }
}

}  // namespace mg
