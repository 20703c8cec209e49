// HIP kernels of one UGKWP time step for gfx950 (FP64 path and the FP32-transport form).
//
// Order inside a step (paper Sec. 2.3, the four-step particle procedure, and Eq.
// update_macro_variables):
//   k_prim_dt      S0  primitives, tau = mu_ref T^omega / p, min Omega/Lambda     (Sec. 2.4(a))
//   k_cell_prep    S0  dt, exp(-dt/tau), rho^h, sample counts N_sam            (Sec. 2.4(b))
//   scan           exclusive prefix of N_sam -> slots of the new particles
//   k_grad         S1  least-squares gradients and limiters (second order only)
//   k_flux(2)      S2  wave flux F^eq + F^{fr,wave} per face                    (Sec. 2.2, 2.4)
//   k_sample       S3  antithetic Maxwellian pairs, uniform positions; start sums S
//   k_inject       S5  free-stream particles entering through far-field faces
//   k_stream       S4+S5 free-flight time and face-to-face transport; end-cell keys;
//                  particles meeting a diffuse wall stop there and are queued
//   k_stream_wall  S5  diffuse re-emission of the queued particles, rest of their flight
//   k_count        bucket sizes (survivors and collided per end cell), slots of movers
//   scan           exclusive prefix of the bucket sizes
//   k_scatter      bucket the movers and collided particles by end cell
//   k_gather       S6  deterministic order per cell, sums E and W^p, update of W
//   k_finalize     step bookkeeping
//   k_avg_cells,   time averaging for steady states, when turned on        (Sec. 2.4(c))
//   k_avg_fin
// No floating-point atomics: per-cell sums use fixed reduction trees, so a run is bitwise
// reproducible.  Integer atomics only hand out bucket slots and counts; the order inside a
// bucket is then fixed by sorting the source indices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "device_common.hpp"
#include "launch.hpp"

namespace ugkwp {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Whole-line stores of particle records with the non-temporal hint: neither the transport nor
// the gather reads back what it writes, and the next kernel's reads of ~1 GB of records do
// not fit in the L2 (measured: transport and gather 3-5% faster)
typedef unsigned int u32x4_nt __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt(uint4 *p, const uint4 &v) {
    const u32x4_nt x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x4_nt *>(p));
}
constexpr int kWave = 64;
constexpr int kScatterChunks = 8;  // particles per thread in k_scatter
constexpr int kSampleCells = 8;     // consecutive cells per wave in k_sample (meshes of 32768 cells or more)
constexpr int kSampleCellsMin = 32768;
constexpr int kGatherWaves = 1;    // cells (waves) per block in k_gather (2 and 4 are slower in FP32)

// ---------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11); counter = (uid, step, tag<<32|sub, 0),
// key = (seed, 0).
// ---------------------------------------------------------------------------------------
struct U4 {
    uint64_t v[4];
};

// 64 x 64 -> 128-bit product from four 32 x 32 + 64 multiply-adds (v_mad_u64_u32); the low
// half reuses the partial products of the high half
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32), bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    const uint64_t p0 = (uint64_t)al * bl;
    const uint64_t t = (uint64_t)al * bh + (p0 >> 32);
    const uint64_t v = (uint64_t)ah * bl + (t & 0xFFFFFFFFULL);
    hi = (uint64_t)ah * bh + ((t >> 32) + (v >> 32));
    lo = (v << 32) | (p0 & 0xFFFFFFFFULL);
}

__device__ __forceinline__ U4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, hi0, lo0);
        mulhilo64(M1, c2, hi1, lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    U4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// counter (particle id, step, tag << 32 | sub, instance), key (seed, 0)
__device__ __forceinline__ U4 draw(uint64_t seed, uint64_t uid, long long step, int tag, uint32_t sub, int inst) {
    return philox(uid, (uint64_t)step, ((uint64_t)tag << 32) | sub, (uint64_t)inst, seed, 0ULL);
}

// instance of a cell (a single instance needs no table)
__device__ __forceinline__ int inst_of(const Dev &D, int c) { return D.n_inst > 1 ? D.cinst[c] : 0; }

// what the transport of one particle needs from its instance
struct StepCtx {
    unsigned long long seed;
    long long step;
    int inst, max_cross;
};

// uniform in (0, 1), never 0 or 1: FP64 (top 52 bits + 1/2) * 2^-52; FP32 (top 23 bits + 1/2)
// * 2^-23, the leading bits of the same draw
template <typename R>
__device__ __forceinline__ R unif(uint64_t r);
template <>
__device__ __forceinline__ double unif<double>(uint64_t r) {
    return ((double)(r >> 12) + 0.5) * 0x1p-52;
}
template <>
__device__ __forceinline__ float unif<float>(uint64_t r) {
    return ((float)(uint32_t)(r >> 41) + 0.5f) * 0x1p-23f;
}

__device__ __forceinline__ uint64_t make_uid(long long step, int cell, long long k) {
    return (((uint64_t)step & 0x7FFFFULL) << 44) | (((uint64_t)cell & 0xFFFFFFULL) << 20) | ((uint64_t)k & 0xFFFFFULL);
}

// ---------------------------------------------------------------------------------------
// Maxwellian moments in a face frame (R = 1, K = 0), lambda = 1/(2T).
// m[k] = <u_n^k> over the full line (rng 0), u_n > 0 (rng 1) or u_n < 0 (rng -1);
// <u^{k+2}> = U <u^{k+1}> + (k+1)/(2 lambda) <u^k> holds on each half line as well.
// The transport type R is double (plain form) or float (FP32 form).
// ---------------------------------------------------------------------------------------
template <typename R>
struct Prim {
    R rho, un, v, w, lam, T;
    int K;  // internal degrees of freedom (Sec. 2.1): <xi^2> = K / (2 lambda)
};

// temperature of a conservative state with K internal degrees of freedom (R = 1):
// rho E = rho |U|^2 / 2 + (3 + K) rho T / 2
__device__ __forceinline__ double temp_k(const double W[5], int K) {
    return (2.0 / (3.0 + K)) * (W[4] - 0.5 * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]) / W[0]) / W[0];
}

template <typename R>
__device__ __forceinline__ void moments4(int rng, R U, R lam, R m[4]) {
    const R pi = (R)kPi;
    if (rng == 0) {
        m[0] = (R)1;
        m[1] = U;
    } else if (rng > 0) {
        m[0] = (R)0.5 * erfc(-sqrt(lam) * U);
        m[1] = U * m[0] + (R)0.5 * exp(-lam * U * U) / sqrt(pi * lam);
    } else {
        m[0] = (R)0.5 * erfc(sqrt(lam) * U);
        m[1] = U * m[0] - (R)0.5 * exp(-lam * U * U) / sqrt(pi * lam);
    }
    m[2] = U * m[1] + (R)1 / ((R)2 * lam) * m[0];
    m[3] = U * m[2] + (R)2 / ((R)2 * lam) * m[1];
}

// <psi> (H) and <u_n psi> (G) of a unit-density Maxwellian; psi = (1, u_n, v, w, (|u|^2 + xi^2)/2)
template <typename R>
__device__ __forceinline__ void psi_moments(const Prim<R> &p, const R m[4], R H[5], R G[5]) {
    R tr = p.v * p.v + p.w * p.w + (R)1 / p.lam + (R)p.K / ((R)2 * p.lam);
    H[0] = m[0];
    H[1] = m[1];
    H[2] = m[0] * p.v;
    H[3] = m[0] * p.w;
    H[4] = (R)0.5 * (m[2] + m[0] * tr);
    G[0] = m[1];
    G[1] = m[2];
    G[2] = m[1] * p.v;
    G[3] = m[1] * p.w;
    G[4] = (R)0.5 * (m[3] + m[1] * tr);
}

// face frame: t1 = normalise(e_a x n), a = axis of the smallest |n_a| (lowest on ties); t2 = n x t1
template <typename R>
__device__ __forceinline__ void face_frame(const R n[3], R t1[3], R t2[3]) {
    int a = 0;
    if (fabs(n[1]) < fabs(n[a])) a = 1;
    if (fabs(n[2]) < fabs(n[a])) a = 2;
    R e0 = a == 0 ? (R)1 : (R)0, e1 = a == 1 ? (R)1 : (R)0, e2 = a == 2 ? (R)1 : (R)0;
    R c0 = e1 * n[2] - e2 * n[1], c1 = e2 * n[0] - e0 * n[2], c2 = e0 * n[1] - e1 * n[0];
    R l = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    t1[0] = c0 / l;
    t1[1] = c1 / l;
    t1[2] = c2 / l;
    t2[0] = n[1] * t1[2] - n[2] * t1[1];
    t2[1] = n[2] * t1[0] - n[0] * t1[2];
    t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

// primitives of a cell state in the face frame; the energy -> temperature recovery is FP64
template <typename R>
__device__ __forceinline__ Prim<R> to_frame(const double W[5], const R n[3], const R t1[3], const R t2[3], int K) {
    Prim<R> p;
    const double U = W[1] / W[0], V = W[2] / W[0], Z = W[3] / W[0];
    const double T = temp_k(W, K);
    const R u = (R)U, v = (R)V, z = (R)Z;
    p.rho = (R)W[0];
    p.un = u * n[0] + v * n[1] + z * n[2];
    p.v = u * t1[0] + v * t1[1] + z * t1[2];
    p.w = u * t2[0] + v * t2[1] + z * t2[2];
    p.T = (R)T;
    p.lam = (R)1 / ((R)2 * p.T);
    p.K = K;
    return p;
}

// Taylor coefficients (-1)^k/k! and (-1)^k (k-1)/k!, k = 2..24, for the series forms of
//   q1/tau = x - 1 + e^-x   and   (q4 - dt e)/tau = 1 - (1 + x) e^-x.
// For second order also (k = 3..24), with q2, q3, q5 + dt^2 e / 2 = tau^2 x^3 times
//   sum (-1)^k (k-2)/k! x^(k-3),  -sum (-1)^k / k! x^(k-3),  sum (-1)^k (k-1)(k-2)/(2 k!) x^(k-3).
struct QSeries {
    double a[25], b[25], c[25], d[25], e[25];
    float af[25], bf[25], cf[25], df[25], ef[25];
    constexpr QSeries() : a(), b(), c(), d(), e(), af(), bf(), cf(), df(), ef() {
        double f = 1.0;
        for (int k = 1; k <= 24; ++k) {
            f = f * k;
            double s = (k % 2 == 0) ? 1.0 : -1.0;
            a[k] = s / f;
            b[k] = s * (k - 1) / f;
            c[k] = s * (k - 2) / f;
            d[k] = -s / f;
            e[k] = s * (double)((k - 1) * (k - 2)) / (2.0 * f);
            af[k] = (float)a[k];
            bf[k] = (float)b[k];
            cf[k] = (float)c[k];
            df[k] = (float)d[k];
            ef[k] = (float)e[k];
        }
    }
};
__constant__ QSeries kQ = QSeries();

// q1 and q4 - dt e of the time-integrated interface distribution (Eq. of q1..q5), x = dt/tau:
// series below x = 1 (terms x^2..x^24 in FP64, x^2..x^12 in FP32, Horner), closed forms above
template <typename R>
__device__ __forceinline__ void qcoef(R dt, R tau, R &q1, R &q4m) {
    const R x = dt / tau;
    if (x < (R)1) {
        R s1 = (R)0, s4 = (R)0;
        if constexpr (sizeof(R) == 8) {
#pragma unroll
            for (int k = 24; k >= 2; --k) {
                s1 = s1 * x + kQ.a[k];
                s4 = s4 * x + kQ.b[k];
            }
        } else {
#pragma unroll
            for (int k = 12; k >= 2; --k) {
                s1 = s1 * x + kQ.af[k];
                s4 = s4 * x + kQ.bf[k];
            }
        }
        q1 = tau * (s1 * x * x);
        q4m = tau * (s4 * x * x);
    } else {
        const R e = exp(-x);
        q1 = tau * (x - (R)1 + e);
        q4m = tau * ((R)1 - ((R)1 + x) * e);
    }
}

// First-order wave flux between two face-frame states (gks: the wave-only start phase, in which
// no particle is sampled and the waves carry the whole free transport q4 g^h of the hydro part):
//   F = rho0 q1 <u_n psi>_0 + (q4 - dt e) (rhoh_l <u_n psi>_{l,u>0} + rhoh_r <u_n psi>_{r,u<0})
// with g0 from the upwind moments of both sides and tau at the face from g0 plus the
// numerical dissipation C2 |pl - pr| / (pl + pr) dt of Sec. 2.4(d).
// Shakhov model (qsh != 0): the g0 term becomes g0^+ = g0 [1 + (1 - Pr) c.q (|c|^2/T - 5) / (5 p T)],
// whose correction carries, over all velocities, no mass or momentum and the energy flux
// (1 - Pr) q.n for any g0 (Gaussian moments <c_n^2 |c|^2> = 5 T^2, <c_n^2 |c|^4> = 35 T^3): F^eq
// gains q1 qsh in energy, qsh = (1 - Pr) q_f.n with q_f the heat flux at the face (shakhov_qsh).
template <typename R>
__device__ __forceinline__ void flux_pair(const Prim<R> &l, const Prim<R> &r, R hl, R hr, R dt, R mu_ref, R omega,
                                          R c2, bool gks, R qsh, R Ff[5]) {
    R ml[4], mr[4], Hl[5], Gl[5], Hr[5], Gr[5];
    moments4<R>(1, l.un, l.lam, ml);
    moments4<R>(-1, r.un, r.lam, mr);
    psi_moments<R>(l, ml, Hl, Gl);
    psi_moments<R>(r, mr, Hr, Gr);
    R W0[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) W0[k] = l.rho * Hl[k] + r.rho * Hr[k];
    Prim<R> z;
    z.rho = W0[0];
    z.un = W0[1] / W0[0];
    z.v = W0[2] / W0[0];
    z.w = W0[3] / W0[0];
    z.K = l.K;
    z.T = ((R)2 / (R)(3 + z.K)) * (W0[4] - (R)0.5 * (W0[1] * W0[1] + W0[2] * W0[2] + W0[3] * W0[3]) / W0[0]) / W0[0];
    z.lam = (R)1 / ((R)2 * z.T);
    R pl = l.rho * l.T, pr = r.rho * r.T;
    R tau = mu_ref * pow(z.T, omega) / (z.rho * z.T) + c2 * (fabs(pl - pr) / (pl + pr)) * dt;
    R q1, q4m;
    qcoef<R>(dt, tau, q1, q4m);
    if (gks) q4m = q4m + dt * exp(-dt / tau);  // wave-only start: the waves carry all of W^h
    R m0[4], H0[5], G0[5];
    moments4<R>(0, z.un, z.lam, m0);
    psi_moments<R>(z, m0, H0, G0);
#pragma unroll
    for (int k = 0; k < 5; ++k) Ff[k] = q1 * z.rho * G0[k] + q4m * (hl * Gl[k] + hr * Gr[k]);
    if (qsh != (R)0) Ff[4] = Ff[4] + q1 * qsh;
}

// ---------------------------------------------------------------------------------------
// wave reductions with a fixed butterfly (deterministic)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = v + __shfl_xor(v, s);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = v + __shfl_xor(v, s);
    return v;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, s));
    return v;
}

// the step's most crossings of one particle: a block's maximum raises the step's (reset by
// k_prim_dt); the atomic is issued only when it would change it (the value read first only
// grows during the step, so a stale read costs at most an extra atomic)
__device__ __forceinline__ void raise_max_cross(const Dev &D, unsigned m) {
    if (m > *(volatile unsigned *)&D.sc->max_cross) atomicMax(&D.sc->max_cross, m);
}

// Totals over the wave of P[0..4] and C[0..4], lane k < 5 receiving P_k and C_k.  Each total
// is built from the same pairwise additions as wave_sum (partial sums of lanes that differ
// in bit 5, then 4, ..., then 0), so it is bitwise wave_sum's; but at each of the first levels
// a lane keeps half of the values it carries and hands its partner the other half: 13
// exchanges instead of 60.
__device__ __forceinline__ void wave_sum_pc(const double P[5], const double C[5], double &pk, double &ck) {
    const int lane = lane_id();
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
    double x[6];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double send = b5 ? P[k] : C[k];
        const double keep = b5 ? C[k] : P[k];
        x[k] = keep + __shfl_xor(send, 32);
    }
    x[5] = 0.0;  // lanes with bit 5 clear now carry the P partial sums, the others the C ones
    double y[4];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double send = b4 ? x[j] : x[3 + j];
        const double keep = b4 ? x[3 + j] : x[j];
        y[j] = keep + __shfl_xor(send, 16);
    }
    y[3] = 0.0;
    double z[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double send = b3 ? y[j] : y[2 + j];
        const double keep = b3 ? y[2 + j] : y[j];
        z[j] = keep + __shfl_xor(send, 8);
    }
    double q;
    {
        const double send = b2 ? z[0] : z[1];
        const double keep = b2 ? z[1] : z[0];
        q = keep + __shfl_xor(send, 4);
    }
    q = q + __shfl_xor(q, 2);
    q = q + __shfl_xor(q, 1);
    // a lane's total is component 3 b4 + 2 b3 + b2 (combinations above 4, or with b3 and b2
    // both set below bit 4, carry the zero padding): P_0..P_4 sit in lanes 0, 4, 8, 16, 20 and
    // C_k 32 lanes above P_k
    const int src = lane < 3 ? 4 * lane : (lane < 5 ? 4 * lane + 4 : 0);
    pk = __shfl(q, src);
    ck = __shfl(q, src + 32);
}

// ---------------------------------------------------------------------------------------
// S0: primitives, tau, min Omega / Lambda
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_prim_dt(Dev D) {
    __shared__ double smin[256];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Scalars *s = D.sc;
        s->n_sampled = 0;
        s->max_cross = 0u;
        s->n_big = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x < kWallSeg) D.wallq[threadIdx.x] = 0u;
    // partial sums of crossings and wall hits of this step's transport
    if (blockIdx.x == 0 && threadIdx.x < 128) D.spart[threadIdx.x] = 0ULL;
    double r = INFINITY;
    int inst = 0;
    if (c < D.nc) {
        const int nc = D.nc;
        inst = inst_of(D, c);
        const InstP &P = D.ip[inst];
        double rho = D.W[c], m0 = D.W[nc + c], m1 = D.W[2 * nc + c], m2 = D.W[3 * nc + c], E = D.W[4 * nc + c];
        bool bad = !(rho > 0.0) || !isfinite(rho);
        double T = 0.0;
        double U = 0.0, V = 0.0, Z = 0.0;
        if (!bad) {
            U = m0 / rho;
            V = m1 / rho;
            Z = m2 / rho;
            T = (2.0 / (3.0 + D.K)) * (E - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho) / rho;
            bad = !(T > 0.0) || !isfinite(T);
        }
        // geometry loaded with W, before any store
        const double dS0 = D.dS[c], dS1 = D.dS[nc + c], dS2 = D.dS[2 * nc + c], vol = D.vol[c];
        if (bad) {
            atomicOr(&D.sc->err, kErrNonPhys);
            D.tau[c] = 1.0;
        } else {
            D.tau[c] = P.mu_ref * pow(T, P.omega) / (rho * T);
            double cs = 3.0 * sqrt(T);
            double lam = (fabs(U) + cs) * dS0 + (fabs(V) + cs) * dS1 + (fabs(Z) + cs) * dS2;
            r = vol / lam;
        }
    }
    // the min over each instance's cells; a block whose cells straddle two instances
    // reports per cell (positive doubles order as their bit patterns)
    const int cfirst = blockIdx.x * blockDim.x;
    const int clast = min(cfirst + (int)blockDim.x, D.nc) - 1;
    if (D.n_inst > 1 && D.cinst[cfirst] != D.cinst[clast]) {
        if (r < INFINITY && r > 0.0) atomicMin(&D.is[inst].dtmin_bits, (unsigned long long)__double_as_longlong(r));
        return;
    }
    smin[threadIdx.x] = r;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && smin[0] < INFINITY && smin[0] > 0.0)
        atomicMin(&D.is[inst_of(D, cfirst)].dtmin_bits, (unsigned long long)__double_as_longlong(smin[0]));
}

// ---------------------------------------------------------------------------------------
// S0 (cont.): dt, collisionless fraction, hydro density, number of particles to sample
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cell_prep(Dev D) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= D.nc) return;
    const int inst = inst_of(D, c);
    const InstP &P = D.ip[inst];
    const double dt = P.cfl * __longlong_as_double((long long)D.is[inst].dtmin_bits);
    const long long step = D.is[inst].step;
    // every per-cell value loaded before the first store
    const double vol = D.vol[c];
    const double Pm = D.P[c];
    const double rho = D.W[c];
    const double tau = D.tau[c];
    const int nleft = D.nleft[c];
    // bucket counters of this step's transport (survivors ending in c, collided ending in c)
    D.cnt64[c] = 0ULL;
    D.cnt64[D.nc + c] = 0ULL;
    if (c == P.cell0) {
        D.is[inst].dt = dt;
        if (inst == 0) D.sc->dt = dt;
    }
    const double rhop = Pm / vol;
    // the hydro density is a difference of sums; below 1e-12 rho it is roundoff of that
    // subtraction (particles hold all the mass) and counts as zero
    const double rh = rho - rhop;
    const double rhoh = rh > 1e-12 * rho ? rh : 0.0;
    // wave-only start phase: no particle is sampled
    const double e = step < P.gks_steps ? 0.0 : exp(-dt / tau);
    D.rhoh[c] = rhoh;
    D.ec[c] = e;
    const double rhohp = e * rhoh;
    long long ns = 0;
    if (rhohp > 0.0 && rhop + rhohp > 0.0) {
        double r = (0.5 * P.n_ref) * (rhohp / (rhop + rhohp));
        double cr = ceil(r);
        if (!(cr <= 524288.0)) {
            atomicOr(&D.sc->err, kErrCellCount);
        } else {
            ns = 2 * (long long)cr;
            long long need = (long long)P.n_min - nleft;
            if (need > 0) {
                long long ne = 2 * ((need + 1) / 2);
                if (ne > ns) ns = ne;
            }
            if (ns > (1LL << 20)) {
                atomicOr(&D.sc->err, kErrCellCount);
                ns = 0;
            }
        }
    }
    D.nsam[c] = ns;
}

// capacity check of the step: old + sampled + entering must fit
__global__ void k_sample_setup(Dev D) {
    Scalars *s = D.sc;
    const long long nn = D.samoff[D.nc];
    const long long ni = D.nff > 0 ? D.injoff[D.nff] : 0;
    if (s->n_old + nn + ni > D.cap) {
        atomicOr(&s->err, kErrCapacity);
        s->n_new = 0;
        s->n_inj = 0;
    } else {
        s->n_new = nn;
        s->n_inj = ni;
    }
    s->n_sampled = (unsigned long long)s->n_new;
    s->n_injected = (unsigned long long)s->n_inj;
}

// Diffuse isothermal wall (Sec. 2.4(e)), first order at the state l (n out of the domain):
// incoming q1 g + (q4 - dt e) g^h with the cell tau; the wall emits rho_w M(T_w, U_w) over
// u_n < 0 for the step, rho_w from zero net mass flux; the mass component is exactly 0.
template <typename R>
__device__ __forceinline__ void diffuse_flux(const Prim<R> &l, R h, R tau_c, const R n[3], const R t1[3],
                                             const R t2[3], const DevBC &bc, R dt, bool gks, R Ff[5]) {
    R q1, q4m;
    qcoef<R>(dt, tau_c, q1, q4m);
    if (gks) q4m = q4m + dt * exp(-dt / tau_c);
    R ml[4], Hl[5], Gl[5];
    moments4<R>(1, l.un, l.lam, ml);
    psi_moments<R>(l, ml, Hl, Gl);
    R Fin[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Fin[k] = q1 * l.rho * Gl[k] + q4m * h * Gl[k];
    const R uw[3] = {(R)bc.Uw[0], (R)bc.Uw[1], (R)bc.Uw[2]};
    Prim<R> w;
    w.rho = (R)1;
    w.un = uw[0] * n[0] + uw[1] * n[1] + uw[2] * n[2];
    w.v = uw[0] * t1[0] + uw[1] * t1[1] + uw[2] * t1[2];
    w.w = uw[0] * t2[0] + uw[1] * t2[1] + uw[2] * t2[2];
    w.T = (R)bc.Tw;
    w.lam = (R)1 / ((R)2 * w.T);
    w.K = l.K;
    R mw[4], Hw[5], Gw[5];
    moments4<R>(-1, w.un, w.lam, mw);
    psi_moments<R>(w, mw, Hw, Gw);
    const R rhow = -Fin[0] / (dt * Gw[0]);
#pragma unroll
    for (int k = 0; k < 5; ++k) Ff[k] = Fin[k] + dt * rhow * Gw[k];
    Ff[0] = (R)0;
}

// Shakhov term of face f (owner c, neighbour nb), FP64: (1 - Pr) q_f.n with the heat flux at the
// face the mean of the two cells' (a far-field face: the free stream's is zero); walls keep the
// BGK flux (0 here).  0 for Pr = 1.
__device__ __forceinline__ double shakhov_qsh(const Dev &D, const InstP &P, int f, int c, int nb) {
    if (P.pr == 1.0) return 0.0;
    if (nb < 0 && D.bc[-1 - nb].type != 2) return 0.0;
    const int nc = D.nc, nf = D.nf;
    const double qa[3] = {D.qh[c], D.qh[nc + c], D.qh[2 * nc + c]};
    double qb[3] = {0.0, 0.0, 0.0};
    if (nb >= 0) {
        qb[0] = D.qh[nb];
        qb[1] = D.qh[nc + nb];
        qb[2] = D.qh[2 * nc + nb];
    }
    const double qn = (0.5 * (qa[0] + qb[0])) * D.fn[f] + (0.5 * (qa[1] + qb[1])) * D.fn[nf + f] +
                      (0.5 * (qa[2] + qb[2])) * D.fn[2 * nf + f];
    return (1.0 - P.pr) * qn;
}

// ---------------------------------------------------------------------------------------
// S2: wave flux per face, times the area, oriented owner -> neighbour.  Arithmetic in R
// (FP32 form: float), inputs recovered from the FP64 state, result stored in FP64.
// ---------------------------------------------------------------------------------------
template <typename R, int BS>
__global__ void __launch_bounds__(BS) k_flux(Dev D) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= D.nf) return;
    const int nc = D.nc, nf = D.nf;
    const int c = D.fown[f];
    const int inst = inst_of(D, c);
    const InstP &P = D.ip[inst];
    if (P.recon != 0) return;
    const R dt = (R)D.is[inst].dt;
    const R mu = (R)P.mu_ref, om = (R)P.omega, c2 = (R)P.c2;
    const bool gks = D.is[inst].step < P.gks_steps;
    const int nb = D.fnb[f];
    R n[3] = {(R)D.fn[f], (R)D.fn[nf + f], (R)D.fn[2 * nf + f]};
    R t1[3], t2[3];
    face_frame<R>(n, t1, t2);
    double Wl[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Wl[k] = D.W[k * nc + c];
    const Prim<R> l = to_frame<R>(Wl, n, t1, t2, D.K);
    const R qsh = (R)shakhov_qsh(D, P, f, c, nb);
    R Ff[5];
    if (nb >= 0) {
        double Wr[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) Wr[k] = D.W[k * nc + nb];
        const Prim<R> r = to_frame<R>(Wr, n, t1, t2, D.K);
        flux_pair<R>(l, r, (R)D.rhoh[c], (R)D.rhoh[nb], dt, mu, om, c2, gks, qsh, Ff);
    } else {
        const DevBC bc = D.bc[-1 - nb];
        if (bc.type == 0) {
            // specular wall: mirror state, keep only the normal momentum
            Prim<R> g = l;
            g.un = -l.un;
            const R h = (R)D.rhoh[c];
            flux_pair<R>(l, g, h, h, dt, mu, om, c2, gks, (R)0, Ff);
            Ff[0] = (R)0;
            Ff[2] = (R)0;
            Ff[3] = (R)0;
            Ff[4] = (R)0;
        } else if (bc.type == 1) {
            diffuse_flux<R>(l, (R)D.rhoh[c], (R)D.tau[c], n, t1, t2, bc, dt, gks, Ff);
        } else {
            // far field: the free stream as the right state (hydro density = its density)
            const Prim<R> r = to_frame<R>(bc.Winf, n, t1, t2, D.K);
            flux_pair<R>(l, r, (R)D.rhoh[c], (R)bc.Winf[0], dt, mu, om, c2, gks, qsh, Ff);
        }
    }
    const R a = (R)D.farea[f];
    D.Phi[f] = (double)(Ff[0] * a);
#pragma unroll
    for (int d = 0; d < 3; ++d) D.Phi[(1 + d) * nf + f] = (double)((Ff[1] * n[d] + Ff[2] * t1[d] + Ff[3] * t2[d]) * a);
    D.Phi[4 * nf + f] = (double)(Ff[4] * a);
}

// ---------------------------------------------------------------------------------------
// Second order (Sec. 2.2 with slopes and time derivative; Sec. 2.4 for the wave part).
// ---------------------------------------------------------------------------------------

// q1, q2, q3, q4 - dt e, q5 + dt^2 e / 2 (series below x = 1, closed forms above)
template <typename R>
__device__ __forceinline__ void qcoef5(R dt, R tau, R q[5]) {
    const R x = dt / tau;
    if (x < (R)1) {
        R s1 = (R)0, s4 = (R)0, s2 = (R)0, s3 = (R)0, s5 = (R)0;
        constexpr int K = sizeof(R) == 8 ? 24 : 12;
#pragma unroll
        for (int k = K; k >= 2; --k) {
            if constexpr (sizeof(R) == 8) {
                s1 = s1 * x + kQ.a[k];
                s4 = s4 * x + kQ.b[k];
                if (k >= 3) {
                    s2 = s2 * x + kQ.c[k];
                    s3 = s3 * x + kQ.d[k];
                    s5 = s5 * x + kQ.e[k];
                }
            } else {
                s1 = s1 * x + kQ.af[k];
                s4 = s4 * x + kQ.bf[k];
                if (k >= 3) {
                    s2 = s2 * x + kQ.cf[k];
                    s3 = s3 * x + kQ.df[k];
                    s5 = s5 * x + kQ.ef[k];
                }
            }
        }
        q[0] = tau * (s1 * x * x);
        q[3] = tau * (s4 * x * x);
        q[1] = tau * tau * (s2 * x * x * x);
        q[2] = tau * tau * (s3 * x * x * x);
        q[4] = tau * tau * (s5 * x * x * x);
    } else {
        const R e = exp(-x);
        q[0] = tau * (x - (R)1 + e);
        q[3] = tau * ((R)1 - ((R)1 + x) * e);
        q[1] = tau * tau * ((R)2 * ((R)1 - e) - x * ((R)1 + e));
        q[2] = tau * tau * ((R)0.5 * x * x - x + (R)1 - e);
        q[4] = tau * tau * (((R)1 + x + (R)0.5 * x * x) * e - (R)1);
    }
}

// <u^k>, k < N, over a range (0 all, +1 u > 0, -1 u < 0)
template <typename R, int N>
__device__ __forceinline__ void moments_n(int rng, R U, R lam, R m[N]) {
    R m4[4];
    moments4<R>(rng, U, lam, m4);
    m[0] = m4[0];
    m[1] = m4[1];
#pragma unroll
    for (int k = 0; k + 2 < N; ++k) m[k + 2] = U * m[k + 1] + (R)(k + 1) / ((R)2 * lam) * m[k];
}

// normal moments over a range to order 6, tangential ones over the full line to order 5, and
// of the K internal components: x2 = <xi^2> = K / (2 lambda), x4 = <xi^4> = K (K + 2) / (4 lambda^2)
template <typename R>
struct Mom3 {
    R u[7], v[6], w[6];
    R x2, x4;
};
template <typename R>
__device__ __forceinline__ void mom3(int rng, const Prim<R> &g, Mom3<R> &M) {
    moments_n<R, 7>(rng, g.un, g.lam, M.u);
    moments_n<R, 6>(0, g.v, g.lam, M.v);
    moments_n<R, 6>(0, g.w, g.lam, M.w);
    M.x2 = (R)g.K / ((R)2 * g.lam);
    M.x4 = (R)(g.K * (g.K + 2)) / ((R)4 * g.lam * g.lam);
}
template <int I, int J, int K, typename R>
__device__ __forceinline__ R mono(const Mom3<R> &M) {
    return M.u[I] * M.v[J] * M.w[K];
}
// < u^I v^J w^K (a . psi) >, a . psi = a0 + a1 u + a2 v + a3 w + a4 (u^2 + v^2 + w^2 + xi^2) / 2
template <int I, int J, int K, typename R>
__device__ __forceinline__ R amom(const Mom3<R> &M, const R a[5]) {
    return a[0] * mono<I, J, K>(M) + a[1] * mono<I + 1, J, K>(M) + a[2] * mono<I, J + 1, K>(M) +
           a[3] * mono<I, J, K + 1>(M) +
           (R)0.5 * a[4] * (mono<I + 2, J, K>(M) + mono<I, J + 2, K>(M) + mono<I, J, K + 2>(M) + mono<I, J, K>(M) * M.x2);
}
// < u^I v^J w^K (a . psi) xi^2 > (the xi components are independent of u, v, w)
template <int I, int J, int K, typename R>
__device__ __forceinline__ R amom_xi(const Mom3<R> &M, const R a[5]) {
    return M.x2 * (a[0] * mono<I, J, K>(M) + a[1] * mono<I + 1, J, K>(M) + a[2] * mono<I, J + 1, K>(M) +
                   a[3] * mono<I, J, K + 1>(M) +
                   (R)0.5 * a[4] * (mono<I + 2, J, K>(M) + mono<I, J + 2, K>(M) + mono<I, J, K + 2>(M))) +
           (R)0.5 * a[4] * mono<I, J, K>(M) * M.x4;
}
// out_k = < u^P v^Q w^S (a . psi) psi_k >
template <int P, int Q, int S, typename R>
__device__ __forceinline__ void gvec(const Mom3<R> &M, const R a[5], R out[5]) {
    out[0] = amom<P, Q, S>(M, a);
    out[1] = amom<P + 1, Q, S>(M, a);
    out[2] = amom<P, Q + 1, S>(M, a);
    out[3] = amom<P, Q, S + 1>(M, a);
    out[4] = (R)0.5 * (amom<P + 2, Q, S>(M, a) + amom<P, Q + 2, S>(M, a) + amom<P, Q, S + 2>(M, a) +
                       amom_xi<P, Q, S>(M, a));
}
// out_k = < u psi_k >
template <typename R>
__device__ __forceinline__ void uvec(const Mom3<R> &M, R out[5]) {
    out[0] = mono<1, 0, 0>(M);
    out[1] = mono<2, 0, 0>(M);
    out[2] = mono<1, 1, 0>(M);
    out[3] = mono<1, 0, 1>(M);
    out[4] = (R)0.5 * (mono<3, 0, 0>(M) + mono<1, 2, 0>(M) + mono<1, 0, 2>(M) + mono<1, 0, 0>(M) * M.x2);
}

// micro slope a with <(a . psi) psi> = b over the unit Maxwellian g, N = 3 + K:
//   R = 2 b5 - (|U|^2 + N/(2 lambda)) b1, R_i = b_{i+1} - U_i b1, a5 = 4 lambda^2/N (R - 2 U.R_i),
//   a_{i+1} = 2 lambda R_i - U_i a5, a1 = b1 - U.a_{2..4} - a5 (|U|^2 + N/(2 lambda))/2
template <typename R>
__device__ __forceinline__ void slope(const Prim<R> &g, const R b[5], R a[5]) {
    const R U0 = g.un, U1 = g.v, U2 = g.w, lam = g.lam;
    const R N = (R)(3 + g.K);
    const R q2 = U0 * U0 + U1 * U1 + U2 * U2;
    const R th = N / ((R)2 * lam);
    const R Rr = (R)2 * b[4] - (q2 + th) * b[0];
    const R R0 = b[1] - U0 * b[0], R1 = b[2] - U1 * b[0], R2 = b[3] - U2 * b[0];
    a[4] = ((R)4 * lam * lam / N) * (Rr - (R)2 * (U0 * R0 + U1 * R1 + U2 * R2));
    a[1] = (R)2 * lam * R0 - U0 * a[4];
    a[2] = (R)2 * lam * R1 - U1 * a[4];
    a[3] = (R)2 * lam * R2 - U2 * a[4];
    a[0] = b[0] - (U0 * a[1] + U1 * a[2] + U2 * a[3]) - (R)0.5 * a[4] * (q2 + th);
}
template <typename R>
__device__ __forceinline__ void slope_of(const Prim<R> &g, const R dW[5], R a[5]) {
    R b[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = dW[k] / g.rho;
    slope<R>(g, b, a);
}

// one side of a face in the face frame: reconstructed state and hydro state with their
// derivatives along n, t1, t2 (hydro density 0: no hydro part)
template <typename R>
struct Side2 {
    Prim<R> g, h;
    R dW[3][5], dWh[3][5];
};

// derivatives of a conservative state along n, t1, t2 from its gradient (G at [3k+d] of a
// [15][stride] array), in frame components
template <typename R>
__device__ __forceinline__ void frame_derivs(const double *G, long long stride, long long idx, const R n[3],
                                             const R t1[3], const R t2[3], R out[3][5]) {
    R g[5][3];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = (R)G[(3 * k + d) * stride + idx];
    const R *e[3] = {n, t1, t2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R dk[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) dk[k] = g[k][0] * e[d][0] + g[k][1] * e[d][1] + g[k][2] * e[d][2];
        out[d][0] = dk[0];
        out[d][1] = dk[1] * n[0] + dk[2] * n[1] + dk[3] * n[2];
        out[d][2] = dk[1] * t1[0] + dk[2] * t1[1] + dk[3] * t1[2];
        out[d][3] = dk[1] * t2[0] + dk[2] * t2[1] + dk[3] * t2[2];
        out[d][4] = dk[4];
    }
}

// second-order flux between two sides (face frame), per unit area:
//   W0 from the upwind half moments; side slopes; abar_d from W_x = rho_l <(a_l . psi) psi>_{>0}
//   + rho_r <(a_r . psi) psi>_{<0}; Abar from <(u abar_n + v abar_t1 + w abar_t2 + Abar) . psi psi> = 0;
//   F = rho0 [q1 <u psi> + q2 <u (u.abar) psi> + q3 <u Abar psi>]
//     + sum_s rho^h_s [(q4 - dt e) <u psi>_s + (q5 + dt^2 e/2) <u (u.a~_s) psi>_s]
// (Shakhov model: + q1 qsh in energy, as in flux_pair)
template <typename R>
__device__ void flux2_pair(const Side2<R> &L, const Side2<R> &Rs, R dt, R mu_ref, R omega, R c2, bool gks, R qsh,
                           R Ff[5]) {
    Mom3<R> ML, MR, M0;
    mom3<R>(1, L.g, ML);
    mom3<R>(-1, Rs.g, MR);
    R W0[5];
    {
        const R one[5] = {(R)1, (R)0, (R)0, (R)0, (R)0};
        R Hl[5], Hr[5];
        gvec<0, 0, 0, R>(ML, one, Hl);
        gvec<0, 0, 0, R>(MR, one, Hr);
#pragma unroll
        for (int k = 0; k < 5; ++k) W0[k] = L.g.rho * Hl[k] + Rs.g.rho * Hr[k];
    }
    Prim<R> z;
    z.rho = W0[0];
    z.un = W0[1] / W0[0];
    z.v = W0[2] / W0[0];
    z.w = W0[3] / W0[0];
    z.K = L.g.K;
    z.T = ((R)2 / (R)(3 + z.K)) * (W0[4] - (R)0.5 * (W0[1] * W0[1] + W0[2] * W0[2] + W0[3] * W0[3]) / W0[0]) / W0[0];
    z.lam = (R)1 / ((R)2 * z.T);
    mom3<R>(0, z, M0);
    R abar[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R al[5], ar[5], Sl[5], Sr[5], Wx[5];
        slope_of<R>(L.g, L.dW[d], al);
        slope_of<R>(Rs.g, Rs.dW[d], ar);
        gvec<0, 0, 0, R>(ML, al, Sl);
        gvec<0, 0, 0, R>(MR, ar, Sr);
#pragma unroll
        for (int k = 0; k < 5; ++k) Wx[k] = L.g.rho * Sl[k] + Rs.g.rho * Sr[k];
        slope_of<R>(z, Wx, abar[d]);
    }
    R At[5];
    {
        R t0[5], t1[5], t2[5], bt[5];
        gvec<1, 0, 0, R>(M0, abar[0], t0);
        gvec<0, 1, 0, R>(M0, abar[1], t1);
        gvec<0, 0, 1, R>(M0, abar[2], t2);
#pragma unroll
        for (int k = 0; k < 5; ++k) bt[k] = -(t0[k] + t1[k] + t2[k]);
        slope<R>(z, bt, At);
    }
    const R pl = L.g.rho * L.g.T, pr = Rs.g.rho * Rs.g.T;
    const R tau = mu_ref * pow(z.T, omega) / (z.rho * z.T) + c2 * (fabs(pl - pr) / (pl + pr)) * dt;
    R q[5];
    qcoef5<R>(dt, tau, q);
    if (gks) {
        // wave-only start: q4 = (q4 - dt e) + dt e, q5 = (q5 + dt^2 e / 2) - dt^2 e / 2
        const R e = exp(-dt / tau);
        q[3] = q[3] + dt * e;
        q[4] = q[4] - (R)0.5 * dt * dt * e;
    }
    {
        R G0[5], X0[5], X1[5], X2[5], GA[5];
        uvec<R>(M0, G0);
        gvec<2, 0, 0, R>(M0, abar[0], X0);
        gvec<1, 1, 0, R>(M0, abar[1], X1);
        gvec<1, 0, 1, R>(M0, abar[2], X2);
        gvec<1, 0, 0, R>(M0, At, GA);
#pragma unroll
        for (int k = 0; k < 5; ++k) Ff[k] = z.rho * (q[0] * G0[k] + q[1] * (X0[k] + X1[k] + X2[k]) + q[2] * GA[k]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const Side2<R> &S = s == 0 ? L : Rs;
        if (!(S.h.rho > (R)0)) continue;
        Mom3<R> MH;
        mom3<R>(s == 0 ? 1 : -1, S.h, MH);
        R ah[5], Gh[5], Y[5], acc[5];
        uvec<R>(MH, Gh);
        slope_of<R>(S.h, S.dWh[0], ah);
        gvec<2, 0, 0, R>(MH, ah, acc);
        slope_of<R>(S.h, S.dWh[1], ah);
        gvec<1, 1, 0, R>(MH, ah, Y);
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += Y[k];
        slope_of<R>(S.h, S.dWh[2], ah);
        gvec<1, 0, 1, R>(MH, ah, Y);
#pragma unroll
        for (int k = 0; k < 5; ++k) Ff[k] += S.h.rho * (q[3] * Gh[k] + q[4] * (acc[k] + Y[k]));
    }
    if (qsh != (R)0) Ff[4] = Ff[4] + q[0] * qsh;
}


// Gradients for second order, one cell per thread, FP64 in both forms: the unweighted
// least-squares gradient over the face neighbours of the 5 components of W and of the hydro
// state (rho^h / rho) W; boundary ghosts at the centre mirrored in the face plane (specular:
// mirror state; diffuse: the cell's density and temperature, velocity reflected about the
// wall's; far field: the free stream); a limiter per component (Barth-Jespersen or
// Venkatakrishnan with eps^2 = (K h)^3, h = Omega^(1/3)); a cell whose limited face states are
// non-physical (rho <= 0, T <= 0, hydro density < 0 or hydro temperature <= 0) falls back to
// first order; a face hydro density within 1e-12 of the face density of zero counts as zero
// (roundoff of an empty hydro part, which the limiter can pin to a neighbour's zero).
__global__ void __launch_bounds__(128) k_grad(Dev D) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= D.nc) return;
    const int nc = D.nc;
    const InstP &P = D.ip[inst_of(D, c)];
    if (P.recon == 0) return;
    double vc[10];
    const double fc = D.rhoh[c] / D.W[c];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        vc[k] = D.W[k * nc + c];
        vc[5 + k] = fc * vc[k];
    }
    const double xc[3] = {D.xc[c], D.xc[nc + c], D.xc[2 * nc + c]};
    double A00 = 0, A01 = 0, A02 = 0, A11 = 0, A12 = 0, A22 = 0;
    double r[10][3], vmax[10], vmin[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        r[k][0] = r[k][1] = r[k][2] = 0.0;
        vmax[k] = vmin[k] = vc[k];
    }
    const int nfc = D.nfc[c];
    for (int lf = 0; lf < nfc; ++lf) {
        const int2 nbl = D.nbl[c * 6 + lf];
        double xj[3], vj[10];
        if (nbl.x >= 0) {
            const int j = nbl.x;
            const double fj = D.rhoh[j] / D.W[j];
#pragma unroll
            for (int d = 0; d < 3; ++d) xj[d] = D.xc[d * nc + j];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                vj[k] = D.W[k * nc + j];
                vj[5 + k] = fj * vj[k];
            }
        } else {
            const double4 pl = D.plane[c * 6 + lf];
            const double nn[3] = {pl.x, pl.y, pl.z};
            const double dist = pl.w - (nn[0] * xc[0] + nn[1] * xc[1] + nn[2] * xc[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) xj[d] = xc[d] + 2.0 * dist * nn[d];
            const DevBC &b = D.bc[-1 - nbl.x];
            if (b.type == 2) {
#pragma unroll
                for (int k = 0; k < 5; ++k) vj[k] = vj[5 + k] = b.Winf[k];
            } else {
                const double rho = vc[0];
                const double U[3] = {vc[1] / rho, vc[2] / rho, vc[3] / rho};
                const double T = temp_k(vc, D.K);
                double Ug[3];
                if (b.type == 0) {
                    const double un = U[0] * nn[0] + U[1] * nn[1] + U[2] * nn[2];
#pragma unroll
                    for (int d = 0; d < 3; ++d) Ug[d] = U[d] - 2.0 * un * nn[d];
                } else {
#pragma unroll
                    for (int d = 0; d < 3; ++d) Ug[d] = 2.0 * b.Uw[d] - U[d];
                }
                vj[0] = rho;
#pragma unroll
                for (int d = 0; d < 3; ++d) vj[1 + d] = rho * Ug[d];
                vj[4] = 0.5 * rho * (Ug[0] * Ug[0] + Ug[1] * Ug[1] + Ug[2] * Ug[2]) + 0.5 * (3.0 + D.K) * rho * T;
#pragma unroll
                for (int k = 0; k < 5; ++k) vj[5 + k] = fc * vj[k];
            }
        }
        const double dx[3] = {xj[0] - xc[0], xj[1] - xc[1], xj[2] - xc[2]};
        A00 += dx[0] * dx[0];
        A01 += dx[0] * dx[1];
        A02 += dx[0] * dx[2];
        A11 += dx[1] * dx[1];
        A12 += dx[1] * dx[2];
        A22 += dx[2] * dx[2];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const double dv = vj[k] - vc[k];
            r[k][0] += dx[0] * dv;
            r[k][1] += dx[1] * dv;
            r[k][2] += dx[2] * dv;
            vmax[k] = fmax(vmax[k], vj[k]);
            vmin[k] = fmin(vmin[k], vj[k]);
        }
    }
    // inverse of the symmetric normal matrix by cofactors
    const double C00 = A11 * A22 - A12 * A12, C01 = A02 * A12 - A01 * A22, C02 = A01 * A12 - A02 * A11;
    const double C11 = A00 * A22 - A02 * A02, C12 = A02 * A01 - A00 * A12, C22 = A00 * A11 - A01 * A01;
    const double det = A00 * C00 + A01 * C01 + A02 * C02;
    double g[10][3];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        g[k][0] = (C00 * r[k][0] + C01 * r[k][1] + C02 * r[k][2]) / det;
        g[k][1] = (C01 * r[k][0] + C11 * r[k][1] + C12 * r[k][2]) / det;
        g[k][2] = (C02 * r[k][0] + C12 * r[k][1] + C22 * r[k][2]) / det;
    }
    const double *lfx = D.lfx + (long long)c * 18;
    {
        const double h = cbrt(D.vol[c]);
        const double kh = P.venkat_k * h;
        const double eps2 = kh * kh * kh;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            double phi = 1.0;
            for (int lf = 0; lf < nfc; ++lf) {
                const double Dk = g[k][0] * (lfx[3 * lf] - xc[0]) + g[k][1] * (lfx[3 * lf + 1] - xc[1]) +
                                  g[k][2] * (lfx[3 * lf + 2] - xc[2]);
                double pf = 1.0;
                if (Dk != 0.0) {
                    const double M = Dk > 0.0 ? vmax[k] - vc[k] : vmin[k] - vc[k];
                    if (P.recon == 1)
                        pf = fmin(1.0, M / Dk);
                    else
                        pf = ((M * M + eps2) * Dk + 2.0 * Dk * Dk * M) / (Dk * (M * M + 2.0 * Dk * Dk + M * Dk + eps2));
                }
                phi = fmin(phi, pf);
            }
            g[k][0] *= phi;
            g[k][1] *= phi;
            g[k][2] *= phi;
        }
    }
    bool ok = true;
    for (int lf = 0; lf < nfc; ++lf) {
        double wf[10];
#pragma unroll
        for (int k = 0; k < 10; ++k)
            wf[k] = vc[k] + g[k][0] * (lfx[3 * lf] - xc[0]) + g[k][1] * (lfx[3 * lf + 1] - xc[1]) +
                    g[k][2] * (lfx[3 * lf + 2] - xc[2]);
        if (!(wf[0] > 0.0) || !(temp_k(wf, D.K) > 0.0)) ok = false;
        if (!(wf[5] >= -1e-12 * wf[0])) ok = false;
        if (wf[5] > 1e-12 * wf[0] && !(temp_k(wf + 5, D.K) > 0.0)) ok = false;
    }
    // every store after the last load (a load issued after a store waits for it as well)
#pragma unroll
    for (int k = 0; k < 5; ++k) D.Wh[k * nc + c] = vc[5 + k];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            D.gW[(3 * k + d) * nc + c] = ok ? g[k][d] : 0.0;
            D.gH[(3 * k + d) * nc + c] = ok ? g[5 + k][d] : 0.0;
        }
}

// a cell's state (and hydro state) extrapolated to point x, FP64
__device__ __forceinline__ void extrap(const Dev &D, int c, const double x[3], double W[5], double Wh[5]) {
    const int nc = D.nc;
    const double dx[3] = {x[0] - D.xc[c], x[1] - D.xc[nc + c], x[2] - D.xc[2 * nc + c]};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        W[k] = D.W[k * nc + c] + D.gW[(3 * k) * nc + c] * dx[0] + D.gW[(3 * k + 1) * nc + c] * dx[1] +
               D.gW[(3 * k + 2) * nc + c] * dx[2];
        Wh[k] = D.Wh[k * nc + c] + D.gH[(3 * k) * nc + c] * dx[0] + D.gH[(3 * k + 1) * nc + c] * dx[1] +
                D.gH[(3 * k + 2) * nc + c] * dx[2];
    }
}

template <typename R>
__device__ __forceinline__ void make_side(const Dev &D, int c, const double W[5], const double Wh[5], const R n[3],
                                          const R t1[3], const R t2[3], Side2<R> &S) {
    S.g = to_frame<R>(W, n, t1, t2, D.K);
    frame_derivs<R>(D.gW, D.nc, c, n, t1, t2, S.dW);
    // a face hydro density at or below 1e-12 of the face density is roundoff of an empty hydro
    // part (the limiter can pin it exactly to a neighbour's zero): no hydro wave on that side
    if (Wh[0] > 1e-12 * W[0]) {
        S.h = to_frame<R>(Wh, n, t1, t2, D.K);
        frame_derivs<R>(D.gH, D.nc, c, n, t1, t2, S.dWh);
    } else {
        S.h.rho = (R)0;
        S.h.K = D.K;
    }
}

// S2 at second order: per face, states extrapolated to the face centre from both sides
// (limited gradients), the flux of flux2_pair; specular walls mirror the reconstructed field
// (derivatives along n and the normal momentum flip), diffuse walls stay first order at the
// reconstructed face state, far-field faces see the free stream with zero gradients.
template <typename R, int BS>
__global__ void __launch_bounds__(BS) k_flux2(Dev D) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= D.nf) return;
    const int nf = D.nf;
    const int c = D.fown[f];
    const int inst = inst_of(D, c);
    const InstP &P = D.ip[inst];
    if (P.recon == 0) return;
    const R dt = (R)D.is[inst].dt;
    const R mu = (R)P.mu_ref, om = (R)P.omega, c2 = (R)P.c2;
    const bool gks = D.is[inst].step < P.gks_steps;
    const int nb = D.fnb[f];
    R n[3] = {(R)D.fn[f], (R)D.fn[nf + f], (R)D.fn[2 * nf + f]};
    R t1[3], t2[3];
    face_frame<R>(n, t1, t2);
    const double xf[3] = {D.fx[f], D.fx[nf + f], D.fx[2 * nf + f]};
    double Wl[5], Whl[5];
    extrap(D, c, xf, Wl, Whl);
    Side2<R> L, Rs;
    make_side<R>(D, c, Wl, Whl, n, t1, t2, L);
    const R qsh = (R)shakhov_qsh(D, P, f, c, nb);
    R Ff[5];
    if (nb >= 0) {
        double Wr[5], Whr[5];
        extrap(D, nb, xf, Wr, Whr);
        make_side<R>(D, nb, Wr, Whr, n, t1, t2, Rs);
        flux2_pair<R>(L, Rs, dt, mu, om, c2, gks, qsh, Ff);
    } else {
        const DevBC bc = D.bc[-1 - nb];
        if (bc.type == 0) {
            Rs = L;
            Rs.g.un = -L.g.un;
            Rs.h.un = -L.h.un;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const R sg = ((d == 0) != (k == 1)) ? (R)-1 : (R)1;
                    Rs.dW[d][k] = sg * L.dW[d][k];
                    Rs.dWh[d][k] = sg * L.dWh[d][k];
                }
            flux2_pair<R>(L, Rs, dt, mu, om, c2, gks, (R)0, Ff);
            Ff[0] = (R)0;
            Ff[2] = (R)0;
            Ff[3] = (R)0;
            Ff[4] = (R)0;
        } else if (bc.type == 1) {
            diffuse_flux<R>(L.g, (R)(Whl[0] > 1e-12 * Wl[0] ? Whl[0] : 0.0), (R)D.tau[c], n, t1, t2, bc, dt, gks,
                            Ff);
        } else {
            Rs.g = to_frame<R>(bc.Winf, n, t1, t2, D.K);
            Rs.h = Rs.g;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int k = 0; k < 5; ++k) Rs.dW[d][k] = Rs.dWh[d][k] = (R)0;
            flux2_pair<R>(L, Rs, dt, mu, om, c2, gks, qsh, Ff);
        }
    }
    const R a = (R)D.farea[f];
    D.Phi[f] = (double)(Ff[0] * a);
#pragma unroll
    for (int d = 0; d < 3; ++d) D.Phi[(1 + d) * nf + f] = (double)((Ff[1] * n[d] + Ff[2] * t1[d] + Ff[3] * t2[d]) * a);
    D.Phi[4 * nf + f] = (double)(Ff[4] * a);
}

// particle store access for the two forms
__device__ __forceinline__ void store_new(const Particles &pa, long long i, const double x[3], const double u[3],
                                          double m, uint64_t uid) {
    double2 *r = reinterpret_cast<double2 *>(pa.rec + i);
    r[0] = make_double2(x[0], x[1]);
    r[1] = make_double2(x[2], u[0]);
    r[2] = make_double2(u[1], u[2]);
    r[3] = make_double2(m, __longlong_as_double((long long)uid));
}
__device__ __forceinline__ void store_new(const Particles &pa, long long i, const float x[3], const float u[3],
                                          float m, uint64_t uid) {
    float4 *r = reinterpret_cast<float4 *>(pa.rec32 + i);
    r[0] = make_float4(x[0], x[1], x[2], u[0]);
    r[1] = make_float4(u[1], u[2], __uint_as_float((uint32_t)uid), __uint_as_float((uint32_t)(uid >> 32)));
    pa.m32[i] = m;
}

// phi = m (1, u, |u|^2 / 2) of a stored particle, accumulated in FP64
template <typename R>
__device__ __forceinline__ void add_phi(double acc[5], R m_, const R u_[3], R e_ = (R)0) {
    const double m = (double)m_, u0 = (double)u_[0], u1 = (double)u_[1], u2 = (double)u_[2], e = (double)e_;
    acc[0] += m;
    acc[1] += m * u0;
    acc[2] += m * u1;
    acc[3] += m * u2;
    acc[4] += m * (0.5 * (u0 * u0 + u1 * u1 + u2 * u2 + e));
}

// internal energy variable e = T |X|^2 of a particle in equilibrium at temperature T: the first K
// of the standard normals that Box-Muller makes of the draws (seed, uid, step, tag, sub0 + j,
// inst), j = 0, 1 (four per draw)
template <typename R>
__device__ __forceinline__ R internal_energy(uint64_t seed, uint64_t uid, long long step, int tag, uint32_t sub0,
                                             int inst, int K, R T) {
    const R two_pi = (R)2 * (R)kPi;
    R acc = (R)0;
    for (int j = 0; 4 * j < K; ++j) {
        const U4 r = draw(seed, uid, step, tag, sub0 + (uint32_t)j, inst);
        const R r1 = sqrt((R)-2 * log(unif<R>(r.v[0]))), r2 = sqrt((R)-2 * log(unif<R>(r.v[2])));
        const R a1 = two_pi * unif<R>(r.v[1]), a2 = two_pi * unif<R>(r.v[3]);
        const R X[4] = {r1 * cos(a1), r1 * sin(a1), r2 * cos(a2), r2 * sin(a2)};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (4 * j + i < K) acc = acc + X[i] * X[i];
    }
    return T * acc;
}
__device__ __forceinline__ void store_e(const Particles &pa, long long i, double e) { pa.e64[i] = e; }
__device__ __forceinline__ void store_e(const Particles &pa, long long i, float e) { pa.e32[i] = e; }
__device__ __forceinline__ double load_e(const Particles &pa, long long i, double) { return pa.e64[i]; }
__device__ __forceinline__ float load_e(const Particles &pa, long long i, float) { return pa.e32[i]; }

// Shakhov model (SH): the survivors' raw moments sum m u_i |u|^2 and sum m u_i u_j as well, so
// that the cell's heat flux for the next step, q = (1/Omega) sum m c |c|^2 / 2 with c = u - U
// and U from W^{n+1}, follows from them and P^{n+1} by expanding c = u - U (the particles and
// the state the next step starts from are exactly these)
template <bool SH>
__device__ __forceinline__ void add_heat(double m, double u0, double u1, double u2, double H[9]) {
    if constexpr (SH) {
        const double w = m * (u0 * u0 + u1 * u1 + u2 * u2);
        H[0] += w * u0;
        H[1] += w * u1;
        H[2] += w * u2;
        H[3] += m * u0 * u0;
        H[4] += m * u0 * u1;
        H[5] += m * u0 * u2;
        H[6] += m * u1 * u1;
        H[7] += m * u1 * u2;
        H[8] += m * u2 * u2;
    }
}
// q of one cell from its survivors' raw moments H (summed as above, then over the wave), its
// P^{n+1} and W^{n+1}: lane i < 3 returns component i,
//   sum m c_i |c|^2 = S3_i - 2 sum_j U_j S2_ij - U_i tr S2 + |U|^2 S1_i + 2 U_i (U . S1) - U_i |U|^2 S0
__device__ __forceinline__ double heat_of(const double H[9], const double Wn[5], const double Pv[5], double vol) {
    const int lane = lane_id();
    const double U[3] = {Wn[1] / Wn[0], Wn[2] / Wn[0], Wn[3] / Wn[0]};
    const double tr = H[3] + H[6] + H[8];
    const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const double us1 = U[0] * Pv[1] + U[1] * Pv[2] + U[2] * Pv[3];
    // lane i takes component i (selects, not register-array indexing)
    const double r0 = H[3] * U[0] + H[4] * U[1] + H[5] * U[2];
    const double r1 = H[4] * U[0] + H[6] * U[1] + H[7] * U[2];
    const double r2 = H[5] * U[0] + H[7] * U[1] + H[8] * U[2];
    const double s2u = lane == 0 ? r0 : (lane == 1 ? r1 : r2);
    const double s3 = lane == 0 ? H[0] : (lane == 1 ? H[1] : H[2]);
    const double s1 = lane == 0 ? Pv[1] : (lane == 1 ? Pv[2] : Pv[3]);
    const double ui = lane == 0 ? U[0] : (lane == 1 ? U[1] : U[2]);
    const double t = s3 - 2.0 * s2u - ui * tr + uu * s1 + 2.0 * ui * us1 - ui * uu * Pv[0];
    return 0.5 * t / vol;
}

// ---------------------------------------------------------------------------------------
// Shakhov model: the heat flux of the gas in each cell at the start of the step,
//   q = (1/Omega) sum_k m_k c_k |c_k|^2 / 2,  c_k = u_k - U,  U = (W_1, W_2, W_3) / W_0,
// over the particles the cell holds (the hydro part, a Maxwellian at the cell's U and T,
// carries none).  The gather of every step leaves it for the next one; this kernel computes it
// after the state is set (init_state, import_state), from the raw moments sum m u_i |u|^2 and
// sum m u_i u_j summed exactly as the gather sums them (lane l the particles s0 + l + 64 k, in
// increasing k), so that both give the same bits.  One wave per cell.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void load_um(const Particles &pa, long long i, double u[3], double &m, double) {
    const double2 *r = reinterpret_cast<const double2 *>(pa.rec + i);
    const double2 a = r[1], b = r[2], t = r[3];
    u[0] = a.y;
    u[1] = b.x;
    u[2] = b.y;
    m = t.x;
}
__device__ __forceinline__ void load_um(const Particles &pa, long long i, double u[3], double &m, float) {
    const float4 *r = reinterpret_cast<const float4 *>(pa.rec32 + i);
    const float4 a = r[0], b = r[1];
    u[0] = (double)a.w;
    u[1] = (double)b.x;
    u[2] = (double)b.y;
    m = (double)pa.m32[i];
}

template <typename R>
__global__ void __launch_bounds__(256) k_heat(Dev D, int buf) {
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int c = blockIdx.x * 4 + wave;
    if (c >= D.nc) return;
    const int nc = D.nc;
    const bool sh = D.ip[inst_of(D, c)].pr != 1.0;
    double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (sh) {
        const long long s0 = D.segoff[buf][c], s1 = D.segoff[buf][c + 1];
        const Particles pa = D.pa[buf];
        for (long long i = s0 + lane; i < s1; i += kWave) {
            double u[3], m;
            load_um(pa, i, u, m, R(0));
            add_heat<true>(m, u[0], u[1], u[2], H);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) H[k] = wave_sum(H[k]);
    }
    double Wn[5], Pv[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        Wn[k] = D.W[k * nc + c];
        Pv[k] = D.P[k * nc + c];
    }
    if (lane < 3) D.qh[lane * nc + c] = sh ? heat_of(H, Wn, Pv, D.vol[c]) : 0.0;
}

// ---------------------------------------------------------------------------------------
// S3: hydro particles, one wave per cell, lane l takes the particles l, l + 64, ...  Pair
// (2p, 2p+1) shares X ~ N(0, I) from Box-Muller on the draw keyed by the even partner's id:
// X0, X1 = r1 (cos, sin)(2 pi e1), r1 = sqrt(-2 ln e0), and X2 = r2 cos(2 pi e3), r2 =
// sqrt(-2 ln e2).  The even partner evaluates the first half, the odd one the second (the
// same code on the other two uniforms), and they exchange halves.  Partners get
// U + sqrt(T) X and U - sqrt(T) X, the pair of Sec. 2.4(b), and their own uniform position
// (box: per axis; tetrahedron: Rocchini-Cignoni folding of the unit cube).  With the
// energy-exact variant (sampling = 1, a departure from the paper) the deviations carry one
// factor s per cell, s = sqrt(3 N_pairs / sum_j |X_j|^2): a first pass sums |X|^2 for s and
// keeps each lane's first half for the second.
// S = P + sum of phi over the new particles (fixed tree over the wave).
// ---------------------------------------------------------------------------------------
// this lane's half of its pair's normal: (r cos a, r sin a), r = sqrt(-2 ln e0 or e2),
// a = 2 pi e1 or e3 (odd lanes use only the cosine)
template <typename R>
__device__ __forceinline__ void half_normal(uint64_t seed, uint64_t puid, long long step, int inst, bool odd,
                                            R &h0, R &h1) {
    const R two_pi = (R)2 * (R)kPi;
    const U4 rv = draw(seed, puid, step, kTagVel, 0, inst);
    const R ea = unif<R>(odd ? rv.v[2] : rv.v[0]), eb = unif<R>(odd ? rv.v[3] : rv.v[1]);
    const R r = sqrt((R)-2 * log(ea));
    h0 = r * cos(two_pi * eb);
    h1 = r * sin(two_pi * eb);
}
// a uniform point of a cell from the draw (uid, step, kTagPos): per axis in a box, the unit cube
// folded onto the tetrahedron (Rocchini-Cignoni) in a tetrahedron; org + s e1 + t e2 + w e3
template <typename R>
__device__ __forceinline__ void cell_point(uint64_t seed, uint64_t uid, long long step, int inst, const R org[3],
                                           const R Ed[9], bool tet, R x[3]) {
    const R one = (R)1;
    U4 rp = draw(seed, uid, step, kTagPos, 0, inst);
    R s = unif<R>(rp.v[0]), t = unif<R>(rp.v[1]), w = unif<R>(rp.v[2]);
    if (tet) {
        if (s + t > one) {
            s = one - s;
            t = one - t;
        }
        if (t + w > one) {
            R tmp = w;
            w = one - s - t;
            t = one - tmp;
        } else if (s + t + w > one) {
            R tmp = w;
            w = s + t + w - one;
            s = one - t - tmp;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = org[d] + s * Ed[d] + t * Ed[3 + d] + w * Ed[6 + d];
}

// one cell's ns > 0 new particles by the whole wave in runs of 64 (ns is even, so a pair never
// straddles two runs), and its S
template <typename R, bool KE>
__device__ __forceinline__ void sample_cell(const Dev &D, int buf, int c, long long ns) {
    const int lane = lane_id();
    const int nc = D.nc;
    const Scalars *sc = D.sc;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    {
        const Particles pa = D.pa[buf];
        const long long base = sc->n_old + D.samoff[c];
        const int inst = inst_of(D, c);
        const InstP &P = D.ip[inst];
        const long long step = D.is[inst].step;
        const unsigned long long seed = P.seed;
        const int cl = c - P.cell0;  // ids carry the cell index within the instance
        const double rho = D.W[c], m0 = D.W[nc + c], m1 = D.W[2 * nc + c], m2 = D.W[3 * nc + c], E = D.W[4 * nc + c];
        const R U[3] = {(R)(m0 / rho), (R)(m1 / rho), (R)(m2 / rho)};
        const R T = (R)((2.0 / (3.0 + D.K)) * (E - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho) / rho);
        R sT = sqrt(T);
        const int K = KE ? D.K : 0;  // KE: K > 0 (a compile-time switch, see add_rec)
        // energy-exact variant with internal degrees of freedom: one factor K N_sam / sum_k |X'_k|^2
        // on every particle's internal energy makes the sample's internal energy exact too
        R fint = (R)1;
        if (P.sampling == 1 && K > 0) {
            R se = (R)0;
            for (long long k = lane; k < ns; k += kWave)
                se = se + internal_energy<R>(seed, make_uid(step, cl, k), step, kTagInt, 0, inst, K, (R)1);
            double sd = wave_sum((double)se);
            fint = (R)((double)K * (double)ns / sd);
        }
        const R one = (R)1;
        const bool odd = (lane & 1) != 0;
        const bool exact = P.sampling == 1;
        R f0 = (R)0, f1 = (R)0;  // this lane's half of its first pair's normal (energy-exact pass)
        if (exact) {
            // energy-exact pairs: the pairs carry the momentum exactly; one factor on every
            // thermal deviation of the cell, sqrt(3 N_pairs / sum_j |X_j|^2), makes the energy
            // exact too (a first pass over the pairs' normal draws, summed in FP64)
            double sx2 = 0.0;
            for (long long k = lane; k < ns; k += kWave) {
                R h0, h1;
                half_normal<R>(seed, make_uid(step, cl, k & ~1LL), step, inst, odd, h0, h1);
                if (k == lane) {
                    f0 = h0;
                    f1 = h1;
                }
                const double a = (double)h0, b = (double)h1;
                sx2 += odd ? a * a : a * a + b * b;
            }
            sx2 = wave_sum(sx2);
            sT = (R)((double)sT * sqrt(3.0 * (double)(ns / 2) / sx2));
        }
        const double vol = D.vol[c];
        const R msam = (R)(D.ec[c] * D.rhoh[c] * vol / (double)ns);
        const R org[3] = {(R)D.orig[c], (R)D.orig[nc + c], (R)D.orig[2 * nc + c]};
        R Ed[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) Ed[q] = (R)D.edge[q * nc + c];
        const bool tet = D.ctype[c] == 4;
        // runs of 64 particles (ns is even, so a pair never straddles two runs)
        for (long long k0 = 0; k0 < ns; k0 += kWave) {
            const long long k = k0 + lane;
            R h0 = f0, h1 = f1;
            if ((k0 > 0 || !exact) && k < ns) half_normal<R>(seed, make_uid(step, cl, k & ~1LL), step, inst, odd, h0, h1);
            const R X0 = __shfl(h0, lane & ~1), X1 = __shfl(h1, lane & ~1), X2 = __shfl(h0, lane | 1);
            if (k < ns) {
                const long long i = base + k;
                const uint64_t uid = make_uid(step, cl, k);
                const R sg = odd ? -one : one;
                const R X[3] = {X0, X1, X2};
                R u[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) u[d] = U[d] + sg * (sT * X[d]);
                R x[3];
                cell_point<R>(seed, uid, step, inst, org, Ed, tet, x);
                store_new(pa, i, x, u, msam, uid);
                pa.cell[i] = c;
                R e = (R)0;
                if (K > 0) {
                    e = internal_energy<R>(seed, uid, step, kTagInt, 0, inst, K, T);
                    if (P.sampling == 1) e = e * fint;
                    store_e(pa, i, e);
                }
                add_phi<R>(acc, msam, u, e);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = wave_sum(acc[k]);
    double ak = acc[0];
#pragma unroll
    for (int k = 1; k < 5; ++k)
        if (lane == k) ak = acc[k];
    if (lane < 5) D.S[lane * nc + c] = D.P[lane * nc + c] + ak;
}

// segmented sum over consecutive lanes: lane l of the segment [first, last] receives the sum of
// v over the segment (fixed order: an inclusive scan by doubling offsets, read at `last`)
__device__ __forceinline__ double seg_sum(double v, int first, int last) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double t = __shfl_up(v, (unsigned)o);
        if (lane - o >= first) v = v + t;
    }
    return __shfl(v, last);
}

// Each wave takes G consecutive cells: runs of consecutive cells whose new particles fit in 64
// lanes together are sampled at once, lane by lane in cell order (most cells sample a few
// particles: one wave per cell left most lanes idle).  G = 8 on meshes of 32768 cells or more;
// a smaller mesh would leave most of the chip idle with a wave per 8 cells, and takes G = 1.  A
// cell with more than 64 is k_sample_big's.  A pair's partners sit in neighbouring lanes of
// one cell (every count and prefix is even); the energy-exact factor and S come from
// segmented sums over the cell's lanes.  The arithmetic per particle is that of sample_cell.
template <typename R, int WPB, bool KE, int G>
__global__ void __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(3))) k_sample(Dev D, int buf) {
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int c0 = (blockIdx.x * WPB + wave) * G;
    if (c0 >= D.nc) return;
    const int nc = D.nc;
    const Scalars *sc = D.sc;
    // new particles of the group's cells; -1 marks a lane without a cell of its own (past the
    // mesh) and a cell of an instance that samples one by one (k_sample_gp's, which also writes
    // its S): neither is sampled nor has S written here
    int myns = -1;
    if (lane < G && c0 + lane < nc) {
        const int c = c0 + lane;
        if (D.gp_any && D.ip[inst_of(D, c)].sampling >= 2)
            myns = -1;
        else
            myns = sc->n_new > 0 ? (int)D.nsam[c] : 0;  // even, at most 2^20
    }
    // wave-uniform counts and prefixes (scalar registers)
    int ns[G];
    int pre[G + 1];
    pre[0] = 0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        ns[j] = __builtin_amdgcn_readfirstlane(__shfl(myns, j));
        const int n = ns[j] > 0 ? ns[j] : 0;
        pre[j + 1] = pre[j] + (n <= kWave ? n : kWave + 1);
    }
    // cells without new particles: S = P (the five loads issued before the first store)
    if (lane < G && myns == 0) {
        const int c = c0 + lane;
        double pv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) pv[k] = D.P[k * nc + c];
#pragma unroll
        for (int k = 0; k < 5; ++k) D.S[k * nc + c] = pv[k] + 0.0;
    }
    // cells with more than 64 new particles go to k_sample_big's list (one atomic per wave)
    {
        const bool big = lane < G && myns > kWave;
        const unsigned long long mb = __ballot(big);
        if (mb) {
            const int first = __ffsll((long long)mb) - 1;
            unsigned int at = 0;
            if (lane == first) at = atomicAdd(&D.sc->n_big, (unsigned int)__popcll(mb));
            at = __shfl(at, first);
            const unsigned long long below = lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
            if (big) D.big[at + __popcll(mb & below)] = c0 + lane;
        }
    }
    int g = 0;
    while (g < G) {
        if (c0 + g >= nc) break;
        if (ns[g] > kWave) {
            ++g;  // k_sample_big's
            continue;
        }
        // the longest run [g, h) of cells of at most 64 particles each that fits in 64 lanes
        int h = g + 1;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (j >= h && j == h && c0 + j < nc && ns[j] <= kWave && pre[j + 1] - pre[g] <= kWave) h = j + 1;
        const int nrun = pre[h] - pre[g];
        if (nrun > 0) {
            // this lane's cell j of the run and its particle k there
            int j = g;
#pragma unroll
            for (int jj = 0; jj < G; ++jj)
                if (jj > g && jj < h && pre[jj] - pre[g] <= lane) j = jj;
            const bool act = lane < nrun;
            const int first = act ? pre[j] - pre[g] : lane, last = act ? pre[j + 1] - pre[g] - 1 : lane;
            const long long k = act ? (long long)(lane - first) : 0;
            const long long nsj = act ? (long long)ns[j] : 0;
            const int c = c0 + j;
            double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            const Particles pa = D.pa[buf];
            const int inst = inst_of(D, c);
            const InstP &P = D.ip[inst];
            const long long step = D.is[inst].step;
            const unsigned long long seed = P.seed;
            const int cl = c - P.cell0;
            const bool exact = P.sampling == 1;
            const bool odd = (k & 1) != 0;
            R h0 = (R)0, h1 = (R)0, sT = (R)0, T = (R)0, fint = (R)1;
            R U[3] = {(R)0, (R)0, (R)0};
            const int K = KE ? D.K : 0;
            double sx2 = 0.0, se = 0.0;
            if (act) {
                const double rho = D.W[c], m0 = D.W[nc + c], m1 = D.W[2 * nc + c], m2 = D.W[3 * nc + c],
                             E = D.W[4 * nc + c];
                U[0] = (R)(m0 / rho);
                U[1] = (R)(m1 / rho);
                U[2] = (R)(m2 / rho);
                T = (R)((2.0 / (3.0 + D.K)) * (E - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho) / rho);
                sT = sqrt(T);
                half_normal<R>(seed, make_uid(step, cl, k & ~1LL), step, inst, odd, h0, h1);
                const double a = (double)h0, b = (double)h1;
                sx2 = odd ? a * a : a * a + b * b;
                if (exact && K > 0) se = (double)internal_energy<R>(seed, make_uid(step, cl, k), step, kTagInt, 0, inst, K, (R)1);
            }
            // energy-exact pairs: one factor per cell on every thermal deviation, sqrt(3 N_pairs /
            // sum_j |X_j|^2), and (K > 0) K N_sam / sum_k |X'_k|^2 on every internal energy
            sx2 = seg_sum(sx2, first, last);
            if (KE) se = seg_sum(se, first, last);
            if (act && exact) {
                sT = (R)((double)sT * sqrt(3.0 * (double)(nsj / 2) / sx2));
                if (K > 0) fint = (R)((double)K * (double)nsj / se);
            }
            const R X0 = __shfl(h0, lane & ~1), X1 = __shfl(h1, lane & ~1), X2 = __shfl(h0, lane | 1);
            if (act) {
                const long long base = sc->n_old + D.samoff[c];
                const R msam = (R)(D.ec[c] * D.rhoh[c] * D.vol[c] / (double)nsj);
                const R org[3] = {(R)D.orig[c], (R)D.orig[nc + c], (R)D.orig[2 * nc + c]};
                R Ed[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) Ed[q] = (R)D.edge[q * nc + c];
                const bool tet = D.ctype[c] == 4;
                const long long i = base + k;
                const uint64_t uid = make_uid(step, cl, k);
                const R sg = odd ? (R)-1 : (R)1;
                const R X[3] = {X0, X1, X2};
                R u[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) u[d] = U[d] + sg * (sT * X[d]);
                R x[3];
                cell_point<R>(seed, uid, step, inst, org, Ed, tet, x);
                store_new(pa, i, x, u, msam, uid);
                pa.cell[i] = c;
                R e = (R)0;
                if (K > 0) {
                    e = internal_energy<R>(seed, uid, step, kTagInt, 0, inst, K, T);
                    if (exact) e = e * fint;
                    store_e(pa, i, e);
                }
                add_phi<R>(acc, msam, u, e);
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) acc[q] = seg_sum(acc[q], first, last);
            if (act && lane == last) {
                double pv[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) pv[q] = D.P[q * nc + c];
#pragma unroll
                for (int q = 0; q < 5; ++q) D.S[q * nc + c] = pv[q] + acc[q];
            }
        }
        g = h;
    }
}

// The cells with more than 64 new particles, which k_sample listed, one wave each (a launch
// of its own, so that its registers do not add to k_sample's); the waves take the list in a
// grid-stride loop (a cell's particles do not depend on which wave samples it).
template <typename R, bool KE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) k_sample_big(Dev D, int buf) {
    const long long nb = (long long)D.sc->n_big;
    const long long waves = (long long)gridDim.x * 8;
    for (long long k = (long long)blockIdx.x * 8 + (int)(threadIdx.x / kWave); k < nb; k += waves) {
        const int c = D.big[k];
        sample_cell<R, KE>(D, buf, c, D.nsam[c]);
    }
}

// ---------------------------------------------------------------------------------------
// S3 with sampling = 2: hydro particles from the first-order g_p (Sec. 2.3).  With g expanded
// about the state W^n the step starts from, at t = dt,
//   g_p = g(W^n) [1 + alpha p],  alpha = dt e/(1 - e) - tau = dt / expm1(dt/tau) - tau,
// and the first-order correction p of the BGK model written in its Chapman-Enskog form
// (X = (u - U)/sqrt(T), z = e_int/T, G_ij = d_j U_i and grad T from the cell's limited
// gradient of W):
//   p = X_i X_j G_ij - (|X|^2 + z)/(3 + K) div U + ((|X|^2 + z)/2 - (5 + K)/2) sqrt(T) X . grad T / T.
// Acceptance-rejection from one stream of proposals per cell: proposal p draws X by Box-Muller
// on (uid_p, step, kTagGP, 0) (X0, X1 = r1 (cos, sin)(2 pi e1), X2 = r2 cos(2 pi e3)), uid_p the
// id a particle p of the cell would have, and, with K > 0, the internal energy T chi^2_K from
// (uid_p, kTagInt, 0 and 1); it is accepted when eta B < 1 + alpha p, eta the first uniform of
// (uid_p, step, kTagGP, 1) in FP64 and
// B = 1 + |alpha| (16 (sum_ij |G_ij| + |div U|) + ((3 + K) 16 + 5 + K)/2 4 sqrt(T) sum_j |d_j T| / T),
// which bounds |1 + alpha p| wherever every normal is at most 4.  The wave tries proposals
// 64 at a time, and the k-th accepted one (in proposal order) becomes particle k, until the
// cell's ns are accepted or min(64 ns, 2^20) proposals are spent; a particle k still missing
// then takes proposal k.  Unlike a proposal loop per particle, no lane idles while the
// slowest lane of its wave keeps rejecting.  Positions as in k_sample.  One wave per cell;
// S = P + the new sums.
// Sampling 3 takes the same draws from the equilibrium itself (weight 1, B = 1: proposal k is
// particle k).  The Shakhov model (Pr != 1) adds (a.X)(|X|^2 - 5) to the weight and 44 |a| to B.
// ---------------------------------------------------------------------------------------
template <typename R, bool KE>
__global__ void __launch_bounds__(256) k_sample_gp(Dev D, int buf) {
    constexpr double kBox = 4.0;
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int c = blockIdx.x * 4 + wave;
    if (c >= D.nc) return;
    const int nc = D.nc;
    const int inst = inst_of(D, c);
    const InstP &P = D.ip[inst];
    if (P.sampling < 2) return;
    const bool gp = P.sampling == 2, sh = P.pr != 1.0;
    const Scalars *sc = D.sc;
    const long long ns = sc->n_new > 0 ? D.nsam[c] : 0;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (ns > 0) {
        const Particles pa = D.pa[buf];
        const long long base = sc->n_old + D.samoff[c];
        const long long step = D.is[inst].step;
        const unsigned long long seed = P.seed;
        const int cl = c - P.cell0;
        const int K = KE ? D.K : 0;
        const double W[5] = {D.W[c], D.W[nc + c], D.W[2 * nc + c], D.W[3 * nc + c], D.W[4 * nc + c]};
        const double rho = W[0], Ud[3] = {W[1] / rho, W[2] / rho, W[3] / rho};
        const double T = temp_k(W, K);
        // primitive gradients from the limited gradient of W: G[i][j] = d_j U_i, gT[j] = d_j T
        // (sampling 2 only; sampling 3 draws from the equilibrium itself)
        double G[3][3], gT[3], sU = 0.0, divU = 0.0, sTg = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            gT[j] = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) G[i][j] = 0.0;
        }
        double alpha = 0.0, Bgp = 1.0;
        if (gp) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double dr = D.gW[j * nc + c];
                double dU[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) dU[i] = (D.gW[(3 * (1 + i) + j) * nc + c] - Ud[i] * dr) / rho;
                double dT = (D.gW[(12 + j) * nc + c] - W[4] / rho * dr) / rho -
                            (Ud[0] * dU[0] + Ud[1] * dU[1] + Ud[2] * dU[2]);
                dT = 2.0 / (3.0 + K) * dT;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    G[i][j] = dU[i];
                    sU += fabs(dU[i]);
                }
                divU += dU[j];
                gT[j] = dT;
                sTg += fabs(dT);
            }
            const double tau = D.tau[c], dt = D.is[inst].dt;
            alpha = dt / expm1(dt / tau) - tau;
            Bgp = 1.0 + fabs(alpha) * (kBox * kBox * (sU + fabs(divU)) +
                                       0.5 * ((3.0 + K) * kBox * kBox + 5.0 + K) * kBox * sqrt(T) * sTg / T);
        }
        // Shakhov model: g^+ / g = 1 + (a.X)(|X|^2 - 5), a = (1 - Pr) q / (5 rho T^(3/2)) with the
        // cell's heat flux q; 44 |a| bounds the correction on |X| <= 4 (clipped beyond)
        double a[3] = {0.0, 0.0, 0.0}, Bsh = 0.0;
        if (sh) {
            const double fa = (1.0 - P.pr) / (5.0 * W[0] * T * sqrt(T));
#pragma unroll
            for (int d = 0; d < 3; ++d) a[d] = fa * D.qh[d * nc + c];
            Bsh = 44.0 * sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        }
        const double B = Bgp + Bsh;
        const double sqT = sqrt(T);
        const R U[3] = {(R)Ud[0], (R)Ud[1], (R)Ud[2]};
        const R sT = (R)sqT, TR = (R)T;
        const R msam = (R)(D.ec[c] * D.rhoh[c] * D.vol[c] / (double)ns);
        const R org[3] = {(R)D.orig[c], (R)D.orig[nc + c], (R)D.orig[2 * nc + c]};
        R Ed[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) Ed[q] = (R)D.edge[q * nc + c];
        const bool tet = D.ctype[c] == 4;
        const R two_pi = (R)2 * (R)kPi;
        // proposal p of the cell (draws keyed by the id a particle p would have): its velocity,
        // internal energy and whether it is accepted
        auto propose = [&](long long p, R u[3], R &e) -> bool {
            const uint64_t uidp = make_uid(step, cl, p);
            const U4 rv = draw(seed, uidp, step, kTagGP, 0u, inst);
            const R r1 = sqrt((R)-2 * log(unif<R>(rv.v[0]))), r2 = sqrt((R)-2 * log(unif<R>(rv.v[2])));
            const R a1 = two_pi * unif<R>(rv.v[1]), a2 = two_pi * unif<R>(rv.v[3]);
            const R X[3] = {(R)(r1 * cos(a1)), (R)(r1 * sin(a1)), (R)(r2 * cos(a2))};
#pragma unroll
            for (int d = 0; d < 3; ++d) u[d] = U[d] + sT * X[d];
            e = (R)0;
            if (KE && K > 0) e = internal_energy<R>(seed, uidp, step, kTagInt, 0u, inst, K, TR);
            const U4 ra = draw(seed, uidp, step, kTagGP, 1u, inst);
            const double x0 = (double)X[0], x1 = (double)X[1], x2 = (double)X[2];
            double w = 1.0;
            if (gp) {
                const double s2 = x0 * x0 + x1 * x1 + x2 * x2 + (double)e / T;
                const double Xd[3] = {x0, x1, x2};
                double shear = 0.0, xg = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    xg += Xd[i] * gT[i];
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj) shear += Xd[i] * Xd[jj] * G[i][jj];
                }
                const double pw = shear - s2 / (3.0 + K) * divU + (0.5 * s2 - 0.5 * (5.0 + K)) * sqT * xg / T;
                w = 1.0 + alpha * pw;
            }
            if (sh) w = w + (a[0] * x0 + a[1] * x1 + a[2] * x2) * ((x0 * x0 + x1 * x1 + x2 * x2) - 5.0);
            return unif<double>(ra.v[0]) * B < w;
        };
        // particle k: its id, position, record and sums
        auto put = [&](long long k, const R u[3], R e) {
            const uint64_t uid = make_uid(step, cl, k);
            const long long i = base + k;
            R x[3];
            cell_point<R>(seed, uid, step, inst, org, Ed, tet, x);
            store_new(pa, i, x, u, msam, uid);
            pa.cell[i] = c;
            if (KE) store_e(pa, i, e);
            add_phi<R>(acc, msam, u, e);
        };
        // the wave tries 64 proposals at a time; the accepted ones, in proposal order, become the
        // next particles (ballot prefix counts), until ns are accepted or the proposals are spent
        const unsigned long long below = lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
        const long long pmax = 64 * ns < (1LL << 20) ? 64 * ns : (1LL << 20);
        long long cnt = 0;
        for (long long p0 = 0; p0 < pmax && cnt < ns; p0 += kWave) {
            const long long p = p0 + lane;
            R u[3] = {(R)0, (R)0, (R)0}, e = (R)0;
            const bool ok = p < pmax && propose(p, u, e);
            const unsigned long long m = __ballot(ok);
            const long long k = cnt + (long long)__popcll(m & below);
            if (ok && k < ns) put(k, u, e);
            cnt += (long long)__popcll(m);
        }
        // proposals spent: a particle k still missing takes proposal k, accepted or not
        for (long long k = (cnt < ns ? cnt : ns) + lane; k < ns; k += kWave) {
            R u[3], e;
            (void)propose(k, u, e);
            put(k, u, e);
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] = wave_sum(acc[k]);
    double ak = acc[0];
#pragma unroll
    for (int k = 1; k < 5; ++k)
        if (lane == k) ak = acc[k];
    if (lane < 5) D.S[lane * nc + c] = D.P[lane * nc + c] + ak;
}

// ---------------------------------------------------------------------------------------
// S5 (far field): free-stream particles entering through far-field faces.  Outside the
// domain the gas is the free stream W_inf; the part of it that reaches a face without a
// collision in the step, exp(-dt/tau_inf) of its density, crosses the face with the
// one-sided number flux Gamma = sigma (phi(a) + a Phi(a)) (a = U_inf.n_in / sigma, sigma =
// sqrt(T_inf)).  Face of area A on cell Omega: mass exp(-dt/tau_inf) rho_inf Gamma A dt in
// N = ceil(Gamma A dt N_ref / Omega) equal particles, none below a ratio of 1e-9.  Particle
// k: normal speed from the flux-weighted half-Maxwellian, tangential components Gaussian
// about U_inf in the face frame, entry point uniform on the face, entry time uniform in
// the step (drawn again by the transport, which starts it on that face).  Computed in FP64
// in both forms; the FP32 form rounds what it stores.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double npdf(double t) { return exp(-0.5 * t * t) / sqrt(2.0 * kPi); }
__device__ __forceinline__ double ncdf(double t) { return 0.5 * erfc(-t / sqrt(2.0)); }

// z = v_n / sigma has density z phi(z - a) / Z(a) on z > 0, Z(a) = phi(a) + a Phi(a), and
// distribution G(z) = (phi(a) - phi(z - a) + a (Phi(z - a) - Phi(-a))) / Z(a); G(z) = eta by
// 60 bisections of [0, max(a, 0) + 40] (the interval ends below 4e-17 wide)
__device__ double flux_speed(double a, double eta) {
    const double pa = npdf(a), Z = pa + a * ncdf(a), cm = ncdf(-a);
    double lo = 0.0, hi = (a > 0.0 ? a : 0.0) + 40.0;
    for (int it = 0; it < 60; ++it) {
        const double z = 0.5 * (lo + hi);
        const double G = (pa - npdf(z - a) + a * (ncdf(z - a) - cm)) / Z;
        if (G < eta)
            lo = z;
        else
            hi = z;
    }
    return 0.5 * (lo + hi);
}

struct Inflow {
    int c, lf, bf, tri, inst;
    double dt;
    long long N;
    double m, sig, a, vt1, vt2, T;
    double nin[3], t1[3], t2[3];
};

__device__ Inflow inflow_face(const Dev &D, int j) {
    Inflow q;
    const int4 fi = D.ffi[j];
    q.c = fi.x;
    q.inst = inst_of(D, q.c);
    const InstP &P = D.ip[q.inst];
    const double dt = D.is[q.inst].dt;
    q.dt = dt;
    q.lf = fi.y & 0xFF;
    q.tri = fi.y >> 8;
    q.bf = fi.z;
    const DevBC &b = D.bc[fi.w];
    const double rho = b.Winf[0];
    const double Ui[3] = {b.Winf[1] / rho, b.Winf[2] / rho, b.Winf[3] / rho};
    const double T = temp_k(b.Winf, D.K);
    q.T = T;
    const double tau = P.mu_ref * pow(T, P.omega) / (rho * T);
    // wave-only start phase: the free stream enters as waves only
    const double e = D.is[q.inst].step < P.gks_steps ? 0.0 : exp(-dt / tau);
    const double4 pl = D.plane[q.c * 6 + q.lf];  // outward: the particle enters along -n
    q.nin[0] = -pl.x;
    q.nin[1] = -pl.y;
    q.nin[2] = -pl.z;
    face_frame<double>(q.nin, q.t1, q.t2);
    q.sig = sqrt(T);
    const double sd = Ui[0] * q.nin[0] + Ui[1] * q.nin[1] + Ui[2] * q.nin[2];
    q.a = sd / q.sig;
    const double Gam = q.sig * (npdf(q.a) + q.a * ncdf(q.a));
    const double area = D.ffg[10 * j + 9];
    const double r = Gam * area * dt * (double)P.n_ref / D.vol[q.c];
    q.N = 0;
    q.m = 0.0;
    if (e * rho > 0.0 && r >= 1e-9) {
        const double cr = ceil(r);
        q.N = cr <= 1048576.0 ? (long long)cr : -1;
        if (q.N > 0) q.m = (e * rho * Gam * area * dt) / (double)q.N;
    }
    q.vt1 = Ui[0] * q.t1[0] + Ui[1] * q.t1[1] + Ui[2] * q.t1[2];
    q.vt2 = Ui[0] * q.t2[0] + Ui[1] * q.t2[1] + Ui[2] * q.t2[2];
    return q;
}

__global__ void __launch_bounds__(256) k_inject_count(Dev D) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.nff) return;
    const Inflow q = inflow_face(D, j);
    long long n = q.N;
    if (n < 0) {
        atomicOr(&D.sc->err, kErrCellCount);
        n = 0;
    }
    D.ninj[j] = n;
}

// one wave per far-field face, lanes over its particles; they follow the sampled ones
template <typename R>
__global__ void __launch_bounds__(64) k_inject(Dev D, int buf) {
    const int j = blockIdx.x;
    const Scalars *sc = D.sc;
    if (sc->n_inj == 0) return;
    const long long n = D.ninj[j];
    if (n <= 0) return;
    const Inflow q = inflow_face(D, j);
    const long long base = sc->n_old + sc->n_new + D.injoff[j];
    const long long step = D.is[q.inst].step;
    const unsigned long long seed = D.ip[q.inst].seed;
    const Particles pa = D.pa[buf];
    const double *g = D.ffg + 10 * j;
    const double two_pi = 2.0 * kPi;
    for (long long k = lane_id(); k < n; k += kWave) {
        const uint64_t uid = (1ULL << 63) | make_uid(step, q.bf, k);
        const U4 rv = draw(seed, uid, step, kTagInject, 0, q.inst);
        const U4 rp = draw(seed, uid, step, kTagPos, 0, q.inst);
        const double vn = q.sig * flux_speed(q.a, unif<double>(rv.v[0]));
        const double rr = sqrt(-2.0 * log(unif<double>(rv.v[1])));
        const double ang = two_pi * unif<double>(rv.v[2]);
        const double X1 = rr * cos(ang), X2 = rr * sin(ang);
        const double w1 = q.vt1 + q.sig * X1, w2 = q.vt2 + q.sig * X2;
        double p1 = unif<double>(rp.v[0]), p2 = unif<double>(rp.v[1]);
        if (q.tri && p1 + p2 > 1.0) {
            p1 = 1.0 - p1;
            p2 = 1.0 - p2;
        }
        R x[3], u[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = (R)(vn * q.nin[d] + w1 * q.t1[d] + w2 * q.t2[d]);
            x[d] = (R)(g[d] + p1 * g[3 + d] + p2 * g[6 + d]);
        }
        store_new(pa, base + k, x, u, (R)q.m, uid);
        pa.cell[base + k] = q.c;
        if (D.K > 0) store_e(pa, base + k, (R)internal_energy<double>(seed, uid, step, kTagInt, 0, q.inst, D.K, q.T));
    }
}

// ---------------------------------------------------------------------------------------
// S4 + S5: face-to-face transport of one particle for time ts (Sec. 2.3).
// Exit time over the faces with n.u > 0 other than the entry face, clamped at 0, lowest local
// face on a tie; an exit time >= the remaining time keeps the particle in the cell.
// Box hexes take a path that evaluates only the three candidate faces; its arithmetic is
// the plane formula (d - n.x) / (n.u) with n = +-e_d, term by term, so both paths give the
// same bits.  Returns 0 inside (cell updated), 1 escaped through a far-field face, -1 lost.
// ---------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ const R *cell_box(const Dev &D, int c);
template <>
__device__ __forceinline__ const double *cell_box<double>(const Dev &D, int c) {
    return D.box + 6 * c;
}
template <>
__device__ __forceinline__ const float *cell_box<float>(const Dev &D, int c) {
    return D.box32 + 6 * c;
}
template <typename R>
__device__ __forceinline__ R face_far(const Dev &D, int s);
template <>
__device__ __forceinline__ double face_far<double>(const Dev &D, int s) {
    return D.nfar[s];
}
template <>
__device__ __forceinline__ float face_far<float>(const Dev &D, int s) {
    return D.nfar32[s];
}

__device__ __forceinline__ void cell_plane(const Dev &D, int s, double p[4]) {
    const double4 q = D.plane[s];
    p[0] = q.x;
    p[1] = q.y;
    p[2] = q.z;
    p[3] = q.w;
}
__device__ __forceinline__ void cell_plane(const Dev &D, int s, float p[4]) {
    const float4 q = D.plane32[s];
    p[0] = q.x;
    p[1] = q.y;
    p[2] = q.z;
    p[3] = q.w;
}

// diffuse re-emission: u_n = sqrt(-2 T_w ln eta) into the domain, tangential components
// N(U_w, T_w) in the face frame; with K internal degrees of freedom (e != nullptr) the internal
// energy variable leaves in equilibrium at T_w too (full accommodation)
template <typename R>
__device__ __forceinline__ void reemit_diffuse(const DevBC &b, const R n[3], R u[3], uint64_t uid, const StepCtx &sx,
                                               int bounce, R *e = nullptr, int K = 0) {
    U4 r = draw(sx.seed, uid, sx.step, kTagWall, (uint32_t)bounce, sx.inst);
    R t1[3], t2[3];
    face_frame<R>(n, t1, t2);
    const R Tw = (R)b.Tw;
    const R sq = sqrt(Tw);
    const R vn = sqrt((R)-2 * Tw * log(unif<R>(r.v[0])));
    const R rr = sqrt((R)-2 * log(unif<R>(r.v[1])));
    const R a = (R)2 * (R)kPi * unif<R>(r.v[2]);
    const R X1 = rr * cos(a), X2 = rr * sin(a);
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = (R)b.Uw[d] - vn * n[d] + sq * (X1 * t1[d] + X2 * t2[d]);
    if (e) *e = internal_energy<R>(sx.seed, uid, sx.step, kTagWallInt, 2u * (uint32_t)bounce, sx.inst, K, Tw);
}

// Flight of one particle for the time ts from cell `cell`, entered through its local face
// `entry` (-1: none).  Returns 0 (ends inside the domain), 1 (left through a far-field face)
// or -1 (more than max_cross crossings); ncross, nwall and bounce (diffuse re-emissions so
// far, which keys the wall draws) carry on from their values at the call.  With STOP, a
// diffuse wall ends the call with 2: x is then the wall point, u the incoming velocity,
// cell the cell at the wall, entry the wall face and ts the time still to fly; the
// re-emission and the rest of the flight are left to a later call (the wall kernel).
// ct0 >= 0: the start cell's type and, for a box cell, its bounds B0 (loaded by the caller
// together with the particle's other start-cell data, so that the first pass does not
// wait for them).
template <typename R, bool STOP>
__device__ int track(const Dev &D, R x[3], R u[3], int &cell, R &ts, int &entry, uint64_t uid, const StepCtx &sx,
                     int &ncross, int &nwall, int &bounce, int ct0 = -1, const R *B0 = nullptr, R *e = nullptr) {
    // margin of the exact division skip below: well above the rounding of the products
    const R skip = sizeof(R) == 8 ? (R)(1.0 + 1e-12) : (R)(1.0f + 1e-5f);
    int c = cell;
    R trem = ts;
    bool first = ct0 >= 0;
    // bounds of box cell c; on conforming boxes a crossing builds them for the next cell
    R B[6];
    bool haveB = first;
    if (first) {
#pragma unroll
        for (int q = 0; q < 6; ++q) B[q] = B0[q];
    }
    for (;;) {
        R best = (R)INFINITY;
        int bf = -1;
        const int ctc = first ? ct0 : (D.all_box ? 8 : (int)D.ctype[c]);
        if (ctc == 8) {
            if (!haveB) {
                const R *Bg = cell_box<R>(D, c);
#pragma unroll
                for (int q = 0; q < 6; ++q) B[q] = Bg[q];
                haveB = true;
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                // a face at distance a >= |u_d| trem (1 + margin) has a computed exit time
                // >= trem, so it can be neither the minimum nor a crossing: no division
                const R ud = u[d];
                if (ud > (R)0) {
                    const R a = B[3 + d] - x[d];
                    if (2 * d + 1 != entry && !(a >= ud * trem * skip)) {
                        R tt = a / ud;
                        if (tt < (R)0) tt = (R)0;
                        if (tt < best) {
                            best = tt;
                            bf = 2 * d + 1;
                        }
                    }
                } else if (ud < (R)0) {
                    const R a = x[d] - B[d];
                    if (2 * d != entry && !(a >= (-ud) * trem * skip)) {
                        R tt = a / (-ud);
                        if (tt < (R)0) tt = (R)0;
                        if (tt < best) {
                            best = tt;
                            bf = 2 * d;
                        }
                    }
                }
            }
        } else {
            const int nfc = D.nfc[c];
            for (int lf = 0; lf < nfc; ++lf) {
                if (lf == entry) continue;
                R p[4];
                cell_plane(D, c * 6 + lf, p);
                const R un = p[0] * u[0] + p[1] * u[1] + p[2] * u[2];
                if (un > (R)0) {
                    R tt = (p[3] - (p[0] * x[0] + p[1] * x[1] + p[2] * x[2])) / un;
                    if (tt < (R)0) tt = (R)0;
                    if (tt < best) {
                        best = tt;
                        bf = lf;
                    }
                }
            }
        }
        first = false;
        if (bf < 0 || best >= trem) {
            x[0] = x[0] + u[0] * trem;
            x[1] = x[1] + u[1] * trem;
            x[2] = x[2] + u[2] * trem;
            cell = c;
            return 0;
        }
        x[0] = x[0] + u[0] * best;
        x[1] = x[1] + u[1] * best;
        x[2] = x[2] + u[2] * best;
        trem = trem - best;
        if (++ncross > sx.max_cross) {
            cell = c;
            return -1;
        }
        const int2 nb = D.nbl[c * 6 + bf];
        // the far bound of the next box, loaded together with the neighbour
        const R far = D.all_box ? face_far<R>(D, c * 6 + bf) : (R)0;
        if (nb.x >= 0) {
            int ent = nb.y;
            if (ent >= kPeriodicEntry) {
                // periodic face: the particle goes on from the partner face at x + shift
                const DevBC &pb = D.bc[ent / kPeriodicEntry - 1];
                x[0] = x[0] + (R)pb.shift[0];
                x[1] = x[1] + (R)pb.shift[1];
                x[2] = x[2] + (R)pb.shift[2];
                ent = ent % kPeriodicEntry;
                haveB = false;
            } else if (D.all_box) {
                // the neighbour shares the whole face: its bounds along the face's axis are
                // this cell's bound at the face and the far one
                const int d = bf >> 1;
                if (bf & 1) {
                    B[d] = B[3 + d];
                    B[3 + d] = far;
                } else {
                    B[3 + d] = B[d];
                    B[d] = far;
                }
            } else {
                haveB = false;
            }
            entry = ent;
            c = nb.x;
            continue;
        }
        const DevBC &b = D.bc[-1 - nb.x];
        if (b.type == 0) {
            if (ctc == 8) {
                // u - 2 (u.n) n with n = +-e_d flips exactly component d
                const int d = bf >> 1;
                u[d] = -u[d];
            } else {
                R p[4];
                cell_plane(D, c * 6 + bf, p);
                const R un = p[0] * u[0] + p[1] * u[1] + p[2] * u[2];
                u[0] = u[0] - (R)2 * un * p[0];
                u[1] = u[1] - (R)2 * un * p[1];
                u[2] = u[2] - (R)2 * un * p[2];
            }
            entry = bf;
        } else if (b.type == 1) {
            if (STOP) {
                cell = c;
                ts = trem;
                entry = bf;
                return 2;
            }
            R p[4];
            cell_plane(D, c * 6 + bf, p);
            const R n[3] = {p[0], p[1], p[2]};
            reemit_diffuse<R>(b, n, u, uid, sx, bounce, e, D.K);
            ++bounce;
            ++nwall;
            entry = bf;
        } else {
            cell = c;
            return 1;
        }
    }
}

// load / store of the transported state of particle i: position and velocity change in
// place, mass and id (the last 16 bytes of an FP64 record, the last 8 of an FP32 one) are
// read for the id and never rewritten
__device__ __forceinline__ void load_state(const Particles &pa, long long i, double x[3], double u[3], uint64_t &uid) {
    const double2 *rp = reinterpret_cast<const double2 *>(pa.rec + i);
    const double2 r0 = rp[0], r1 = rp[1], r2 = rp[2];
    uid = (uint64_t)__double_as_longlong(reinterpret_cast<const double *>(rp + 3)[1]);
    x[0] = r0.x;
    x[1] = r0.y;
    x[2] = r1.x;
    u[0] = r1.y;
    u[1] = r2.x;
    u[2] = r2.y;
}
__device__ __forceinline__ void store_state(const Particles &pa, long long i, const double x[3], const double u[3]) {
    double2 *rp = reinterpret_cast<double2 *>(pa.rec + i);
    rp[0] = make_double2(x[0], x[1]);
    rp[1] = make_double2(x[2], u[0]);
    rp[2] = make_double2(u[1], u[2]);
}
__device__ __forceinline__ void load_state(const Particles &pa, long long i, float x[3], float u[3], uint64_t &uid) {
    const float4 *rp = reinterpret_cast<const float4 *>(pa.rec32 + i);
    const float4 a = rp[0], b = rp[1];
    x[0] = a.x;
    x[1] = a.y;
    x[2] = a.z;
    u[0] = a.w;
    u[1] = b.x;
    u[2] = b.y;
    uid = (uint64_t)__float_as_uint(b.z) | ((uint64_t)__float_as_uint(b.w) << 32);
}
__device__ __forceinline__ void store_state(const Particles &pa, long long i, const float x[3], const float u[3]) {
    float4 *rp = reinterpret_cast<float4 *>(pa.rec32 + i);
    rp[0] = make_float4(x[0], x[1], x[2], u[0]);
    float2 *q = reinterpret_cast<float2 *>(rp + 1);
    q[0] = make_float2(u[1], u[2]);
}

// Free flight and transport of the particles, ILP particles per thread (their loads are all
// issued before the first is tracked, so that each thread keeps ILP memory chains in flight);
// blocks past the live particles exit at once.  The free-flight time of an old particle is
// t_f = -tau ln eta with tau of its start cell; it collides iff t_f < dt.  Since t_f < dt <=>
// eta > exp(-dt/tau), eta below exp(-dt/tau) by a relative margin decides the comparison
// without the logarithm (the same decision as the formula, which is evaluated near the
// threshold and for every collided particle).
// Key of the end bucket: end cell (stays collisionless), nc + end cell (collided), -1
// (escaped); stayers (collisionless, no face met) carry kStayBit and their records are not
// stored (the gather advances them), nor are those of escaped particles.
// A particle that meets a diffuse wall stops there (its state at the wall is stored) and is
// queued with what its flight still needs (WallCont, kept in the next step's buffer, which
// is free until the gather); the wall kernel re-emits it and finishes the flight with the
// same draws and arithmetic.  The re-emission (logarithm, sine, cosine) is thereby kept out
// of the transport kernel's registers.
template <typename R>
struct WallCont {
    R trem;                   // flight time left at the wall
    int ncross, bounce;       // crossings so far (the wall included), re-emissions so far
    int entry, c0, collided;  // wall face, start cell (-1: entered this step), collided flag
    int cell;                 // cell at the wall
};
static_assert(sizeof(WallCont<double>) <= sizeof(PRec) && sizeof(WallCont<float>) <= sizeof(PRec32),
              "a continuation fits in a particle record");
template <typename R>
__device__ __forceinline__ WallCont<R> *wall_cont(const Particles &p, long long i);
template <>
__device__ __forceinline__ WallCont<double> *wall_cont<double>(const Particles &p, long long i) {
    return reinterpret_cast<WallCont<double> *>(p.rec + i);
}
template <>
__device__ __forceinline__ WallCont<float> *wall_cont<float>(const Particles &p, long long i) {
    return reinterpret_cast<WallCont<float> *>(p.rec32 + i);
}

// end of a flight: state (unless the caller stores it) and bucket key of particle i (the key
// carries the end cell; the cell array of this buffer is not read again, the gather writes
// the next one).  A stayer (kStayBit) flew collisionless for the whole step without meeting
// any face: its state is x + u dt of its record, which the gather forms itself, so its record
// is not rewritten here.  Returns whether the record must be stored (every particle that is
// neither a stayer nor escaped).
template <typename R, bool STORE>
__device__ __forceinline__ bool finish_flight(const Dev &D, const Particles &pa, long long i, const R x[3],
                                              const R u[3], int c, int rc, bool collided, int c0, int ncross,
                                              bool &lost) {
    if (STORE) store_state(pa, i, x, u);
    int key = -1;
    bool stay = false;
    if (rc != 1) {
        lost = lost || rc < 0;
        key = collided ? D.nc + c : c;
        stay = !collided && c == c0 && ncross == 0;
    }
    D.key[i] = stay ? (key | kStayBit) : key;
    return rc != 1 && !stay;
}

template <typename R, bool MULTI, bool STORE>
__device__ __forceinline__ void stream_one(const Dev &D, const Particles &pa, const Particles &pc, long long i,
                                           long long n_old, long long n_smp, int c, R x[3], R u[3], uint64_t uid,
                                           R e, R tauc, unsigned long long &nx_, unsigned &mx_, bool &lost,
                                           bool &queued, bool &wr, int ct0, const R *B0, int inst_c) {
    const R lmargin = sizeof(R) == 8 ? (R)(1.0 - 1e-12) : (R)(1.0f - 1e-5f);
    int c0 = c;
    // a single instance reads its values through uniform addresses
    const int inst = MULTI ? inst_c : 0;
    const InstP &P = D.ip[inst];
    const double dt64 = D.is[inst].dt;
    const R dt = (R)dt64;
    const StepCtx sx{P.seed, D.is[inst].step, inst, P.max_cross};
    R ts = dt;
    int entry0 = -1;
    bool collided = false;
    if (i >= n_smp) {
        // entering through a far-field face: from its entry time to the end of the step,
        // starting on that face; never a stayer (it did not start in a cell)
        const U4 r = draw(sx.seed, uid, sx.step, kTagInject, 0, inst);
        ts = (R)(unif<double>(r.v[3]) * dt64);
        entry0 = D.bflf[P.bf0 + (long long)((uid >> 20) & 0xFFFFFFULL)];
        c0 = -1;
    } else if (i < n_old) {
        const U4 r = draw(sx.seed, uid, sx.step, kTagTF, 0, inst);
        const R eta = unif<R>(r.v[0]);
        if (!(eta < e * lmargin)) {
            const R tf = -tauc * log(eta);
            if (tf < dt) {
                ts = tf;
                collided = true;
            }
        }
    }
    int nx = 0, nw = 0, bounce = 0;
    int entry = entry0;
    const int rc = track<R, true>(D, x, u, c, ts, entry, uid, sx, nx, nw, bounce, ct0, B0);
    nx_ += (unsigned long long)nx;
    if (rc == 2) {  // its count goes on in k_stream_wall
        if (STORE) store_state(pa, i, x, u);
        *wall_cont<R>(pc, i) = WallCont<R>{ts, nx, bounce, entry, c0, collided ? 1 : 0, c};
        queued = true;
        wr = true;
        return;
    }
    mx_ = max(mx_, (unsigned)nx);
    wr = finish_flight<R, STORE>(D, pa, i, x, u, c, rc, collided, c0, nx, lost);
}

// a record as 16-byte chunks
template <typename R>
struct RecChunks;
template <>
struct RecChunks<double> {
    static constexpr int N = 4;  // x0 x1 | x2 u0 | u1 u2 | m id
};
template <>
struct RecChunks<float> {
    static constexpr int N = 2;  // x0 x1 x2 u0 | u1 u2 id
};
__device__ __forceinline__ uint4 *rec_chunks(const Particles &p, long long i, double) {
    return reinterpret_cast<uint4 *>(p.rec + i);
}
__device__ __forceinline__ uint4 *rec_chunks(const Particles &p, long long i, float) {
    return reinterpret_cast<uint4 *>(p.rec32 + i);
}

// the transported state of a lane's particle into its slot of the wave's stage: position and
// velocity with the mass and id chunk (FP64) or id words (FP32) as loaded
__device__ __forceinline__ void stage_state(uint4 *slot, const double x[3], const double u[3], const uint4 &tail) {
    double2 *d = reinterpret_cast<double2 *>(slot);
    d[0] = make_double2(x[0], x[1]);
    d[1] = make_double2(x[2], u[0]);
    d[2] = make_double2(u[1], u[2]);
    slot[3] = tail;
}
__device__ __forceinline__ void stage_state(uint4 *slot, const float x[3], const float u[3], const uint4 &tail) {
    float4 *f = reinterpret_cast<float4 *>(slot);
    f[0] = make_float4(x[0], x[1], x[2], u[0]);
    f[1] = make_float4(u[1], u[2], __uint_as_float(tail.z), __uint_as_float(tail.w));
}
// the last 16 bytes of a record as loaded (FP64: mass and id; FP32: u1 u2 and the id words)
__device__ __forceinline__ uint4 rec_tail(const Particles &pa, long long i, double) {
    return reinterpret_cast<const uint4 *>(pa.rec + i)[3];
}
__device__ __forceinline__ uint4 rec_tail(const Particles &pa, long long i, float) {
    return reinterpret_cast<const uint4 *>(pa.rec32 + i)[1];
}

template <typename R, int BS, bool MULTI, int ILP>
__global__ void __launch_bounds__(BS) k_stream(Dev D, int buf, long long qseg) {
    constexpr int NW = BS / 64;
    constexpr int CPR = RecChunks<R>::N;
    __shared__ unsigned long long red[2][NW];
    // output stage: the records of each wave's run, stored whole and coalesced at the end
    __shared__ uint4 stage[NW][ILP][kWave * CPR];
    const Scalars *sc = D.sc;
    const long long n_old = sc->n_old;
    const long long n_smp = n_old + sc->n_new;
    const long long n_tot = n_smp + sc->n_inj;
    const long long i0 = (long long)blockIdx.x * (BS * ILP);
    if (i0 >= n_tot) return;
    const Particles pa = D.pa[buf], pc = D.pa[buf ^ 1];
    unsigned long long nx_ = 0;
    unsigned mx_ = 0;  // most crossings of one of this lane's particles
    bool lost = false;
    long long ii[ILP];
    int cc[ILP];
    bool qq[ILP], wr[ILP];
    uint4 tl[ILP];
    R xx[ILP][3], uu[ILP][3], ee[ILP], tt[ILP], bx[ILP][6];
    int ct[ILP], ins[ILP];
    uint64_t id[ILP];
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        ii[j] = i0 + j * BS + threadIdx.x;
        if (ii[j] < n_tot) {
            cc[j] = pa.cell[ii[j]];
            load_state(pa, ii[j], xx[j], uu[j], id[j]);
            tl[j] = rec_tail(pa, ii[j], R(0));
        }
    }
    // start-cell data (e, tau, cell type, box bounds, instance), loaded before the generators
    // run, all in one round
#pragma unroll
    for (int j = 0; j < ILP; ++j)
        if (ii[j] < n_tot) {
            ee[j] = (R)D.ec[cc[j]];
            tt[j] = (R)D.tau[cc[j]];
            ct[j] = D.all_box ? 8 : (int)D.ctype[cc[j]];
            ins[j] = MULTI ? D.cinst[cc[j]] : 0;
            const R *Bg = cell_box<R>(D, cc[j]);
#pragma unroll
            for (int q = 0; q < 6; ++q) bx[j][q] = Bg[q];
        }
    unsigned long long wm[ILP];
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        qq[j] = false;
        wr[j] = false;
        if (ii[j] < n_tot) {
            stream_one<R, MULTI, false>(D, pa, pc, ii[j], n_old, n_smp, cc[j], xx[j], uu[j], id[j], ee[j], tt[j], nx_,
                                        mx_, lost, qq[j], wr[j], ct[j], bx[j], ins[j]);
            stage_state(&stage[threadIdx.x / kWave][j][lane_id() * CPR], xx[j], uu[j], tl[j]);
        }
        wm[j] = __ballot(wr[j]);
    }
    // each wave stores the records of its runs that changed (stayers and escaped particles
    // are skipped), consecutive lanes on consecutive chunks
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        const long long wb = i0 + j * BS + (threadIdx.x / kWave) * kWave;  // the run's first record
        const long long nr = n_tot - wb;
        const int nch = (nr <= 0 ? 0 : (nr >= kWave ? kWave : (int)nr)) * CPR;
        uint4 *g = rec_chunks(pa, wb, R(0));
        for (int k = lane_id(); k < nch; k += kWave)
            if ((wm[j] >> (k / CPR)) & 1ULL) st_nt(&g[k], stage[threadIdx.x / kWave][j][k]);
    }
    // wall queue (held in the rank array, which the bucket count fills only later): this
    // block's segment, qseg entries from seg * qseg
    const int lane = lane_id();
    const unsigned long long below = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    const int seg = (int)(blockIdx.x % kWallSeg);
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        const unsigned long long m = __ballot(qq[j]);
        if (m) {
            const int first = __ffsll((long long)m) - 1;
            unsigned int base = 0;
            if (lane == first) base = atomicAdd(&D.wallq[seg], (unsigned int)__popcll(m));
            base = __shfl(base, first);
            if (qq[j]) D.rank[seg * qseg + base + __popcll(m & below)] = (int32_t)ii[j];
        }
    }
    if (__ballot(lost) && lane == 0) atomicOr(&D.sc->err, kErrLost);
    nx_ = wave_sum_u64(nx_);
    mx_ = wave_max_u32(mx_);
    const int wave = threadIdx.x / kWave;
    if (lane == 0) {
        red[0][wave] = nx_;
        red[1][wave] = mx_;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, m = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            a += red[0][w];
            m = max(m, red[1][w]);
        }
        if (a) atomicAdd(&D.spart[blockIdx.x & 63], a);
        raise_max_cross(D, (unsigned)m);
    }
}

// The diffuse re-emissions queued by k_stream and the rest of those flights (further walls
// re-emitted here directly).  Block b serves queue segment b % kWallSeg in a block-stride
// loop together with the other gridDim / kWallSeg blocks of that segment.
template <typename R, bool MULTI, bool KE>
__global__ void __launch_bounds__(256) k_stream_wall(Dev D, int buf, long long qseg) {
    __shared__ unsigned long long red[2][4];
    __shared__ unsigned redm[4];
    const int seg = (int)(blockIdx.x % kWallSeg);
    const long long nq = (long long)D.wallq[seg];
    const long long per = (long long)(gridDim.x / kWallSeg) * 256;
    const Particles pa = D.pa[buf], pc = D.pa[buf ^ 1];
    unsigned long long nx_ = 0, nw_ = 0;
    unsigned mx_ = 0;
    bool lost = false;
    for (long long q = (long long)(blockIdx.x / kWallSeg) * 256 + threadIdx.x; q < nq; q += per) {
        const long long i = D.rank[seg * qseg + q];
        R x[3], u[3];
        uint64_t uid;
        load_state(pa, i, x, u, uid);
        const WallCont<R> w = *wall_cont<R>(pc, i);
        int c = w.cell;
        const int inst = MULTI ? D.cinst[c] : 0;
        const InstP &P = D.ip[inst];
        const StepCtx sx{P.seed, D.is[inst].step, inst, P.max_cross};
        const DevBC &b = D.bc[-1 - D.nbl[c * 6 + w.entry].x];
        R p[4];
        cell_plane(D, c * 6 + w.entry, p);
        const R n[3] = {p[0], p[1], p[2]};
        R ev = (R)0;
        R *ep = KE ? &ev : nullptr;
        reemit_diffuse<R>(b, n, u, uid, sx, w.bounce, ep, KE ? D.K : 0);
        int nx = w.ncross, nw = 1, bounce = w.bounce + 1;
        int entry = w.entry;
        R ts = w.trem;
        const int rc = track<R, false>(D, x, u, c, ts, entry, uid, sx, nx, nw, bounce, -1, nullptr, ep);
        if (ep) store_e(pa, i, ev);
        nx_ += (unsigned long long)(nx - w.ncross);
        nw_ += (unsigned long long)nw;
        mx_ = max(mx_, (unsigned)nx);
        (void)finish_flight<R, true>(D, pa, i, x, u, c, rc, w.collided != 0, w.c0, nx, lost);
    }
    if (__ballot(lost) && lane_id() == 0) atomicOr(&D.sc->err, kErrLost);
    nx_ = wave_sum_u64(nx_);
    nw_ = wave_sum_u64(nw_);
    mx_ = wave_max_u32(mx_);
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) {
        red[0][wave] = nx_;
        red[1][wave] = nw_;
        redm[wave] = mx_;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long a = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const unsigned long long bw = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        const int slot64 = blockIdx.x & 63;
        if (a) atomicAdd(&D.spart[slot64], a);
        if (bw) atomicAdd(&D.spart[64 + slot64], bw);
        raise_max_cross(D, max(max(redm[0], redm[1]), max(redm[2], redm[3])));
    }
}

// Lanes of a wave grouped by key with ballots only: mine = the lanes that share this lane's
// key (0 for key < 0).  Must be called by the whole wave.
__device__ __forceinline__ unsigned long long key_group(int key) {
    unsigned long long todo = __ballot(key >= 0);
    unsigned long long mine = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lkey = __shfl(key, leader);
        const unsigned long long same = __ballot(key == lkey) & todo;
        if (key == lkey) mine = same;
        todo &= ~same;
    }
    return mine;
}

// bucket counts: stayers are only counted, movers and collided particles get their slot in
// the bucket (the order of those slots is fixed later by sorting in the gather).  A block
// takes 4 waves x CH runs of 64 consecutive particles and counts them in an LDS
// hash table keyed by bucket (open addressing, as many entries as the block has particles,
// so it cannot fill up; entry = stayers << 32 | movers).  Stayers are grouped by ballots
// (one LDS atomic per group); a mover or collided particle adds itself, and the returned
// count is its place among the block's particles of that key.  Then one global 64-bit
// atomic per distinct key of the block adds the block's count to the bucket counter and
// returns the block's base.  Particles are sorted by start cell, so a block holds a few
// dozen distinct keys.
template <int CH>
__global__ void __launch_bounds__(256) k_count(Dev D) {
    constexpr int TS = 256 * CH;
    constexpr int LOG_TS = __builtin_ctz(TS);
    static_assert((TS & (TS - 1)) == 0, "hash table size must be a power of two");
    __shared__ int tkey[TS];
    __shared__ unsigned long long tcnt[TS];
    const Scalars *sc = D.sc;
    const long long n_tot = sc->n_old + sc->n_new + sc->n_inj;
    const long long b0 = (long long)blockIdx.x * TS;
    if (b0 >= n_tot) return;
    const int lane = lane_id();
    const long long w0 = b0 + (long long)(threadIdx.x / kWave) * (kWave * CH);
    for (int h = threadIdx.x; h < TS; h += 256) {
        tkey[h] = -1;
        tcnt[h] = 0ULL;
    }
    int key[CH];
    bool stay[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const long long i = w0 + j * kWave + lane;
        const int kraw = i < n_tot ? D.key[i] : -1;
        stay[j] = kraw >= 0 && (kraw & kStayBit) != 0;
        key[j] = kraw >= 0 ? (kraw & ~kStayBit) : -1;
    }
    __syncthreads();
    int slot[CH];
    unsigned int local[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        // stayers (most lanes, usually one or two keys per run): grouped by ballots, each
        // group's leader counts the group in the high word of its key's entry
        const unsigned long long mine = key_group(stay[j] ? key[j] : -1);
        const int leader = mine ? __ffsll((long long)mine) - 1 : lane;
        const bool lead = mine && lane == leader;
        // movers and collided particles (mostly distinct keys within a run): each lane on its
        // own entry, whose low word hands out its place among the block's particles of the key
        slot[j] = -1;
        local[j] = 0;
        if (lead || (key[j] >= 0 && !stay[j])) {
            int sl = -1;
            unsigned int h = ((unsigned int)key[j] * 0x9E3779B1u) >> (32 - LOG_TS);
            for (int probe = 0; probe < TS; ++probe) {
                const int k = atomicCAS(&tkey[h], -1, key[j]);
                if (k == -1 || k == key[j]) {
                    sl = (int)h;
                    break;
                }
                h = (h + 1) & (unsigned int)(TS - 1);
            }
            // always found: distinct keys <= particles of the block = TS
            if (sl < 0) {
                atomicOr(&D.sc->err, kErrLost);
            } else if (stay[j]) {
                atomicAdd(&tcnt[sl], (unsigned long long)__popcll(mine) << 32);
            } else {
                slot[j] = sl;
                local[j] = (unsigned int)(atomicAdd(&tcnt[sl], 1ULL) & 0xFFFFFFFFULL);
            }
        }
    }
    __syncthreads();
    // block totals into the buckets; the entry's count is replaced by the block's base (all
    // of a thread's atomics are issued before the first result is waited for)
    {
        constexpr int PT = TS / 256;
        int hk[PT];
        unsigned long long hv[PT];
#pragma unroll
        for (int q = 0; q < PT; ++q) {
            hk[q] = tkey[q * 256 + threadIdx.x];
            hv[q] = tcnt[q * 256 + threadIdx.x];
        }
#pragma unroll
        for (int q = 0; q < PT; ++q)
            if (hk[q] >= 0) hv[q] = atomicAdd(&D.cnt64[hk[q]], hv[q]);
#pragma unroll
        for (int q = 0; q < PT; ++q)
            if (hk[q] >= 0) tcnt[q * 256 + threadIdx.x] = hv[q];
    }
    __syncthreads();
    unsigned long long base[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) base[j] = tcnt[slot[j] >= 0 ? slot[j] : 0];
#pragma unroll
    for (int j = 0; j < CH; ++j)
        if (key[j] >= 0 && !stay[j] && slot[j] >= 0)
            D.rank[w0 + j * kWave + lane] = (int)(base[j] & 0xFFFFFFFFULL) + (int)local[j];
}

// bucket the movers (collisionless particles that changed cell) and the collided particles:
// perm[off[key] + rank] = i (cnt holds their number per bucket); stayers are collected by
// the gather from their own segment.  kScatterChunks particles per thread, strided by the
// block; their loads are issued before the first store.
__global__ void __launch_bounds__(256) k_scatter(Dev D) {
    constexpr int CH = kScatterChunks;
    const Scalars *sc = D.sc;
    const long long n_tot = sc->n_old + sc->n_new + sc->n_inj;
    const long long b0 = (long long)blockIdx.x * (256 * CH);
    if (b0 >= n_tot) return;
    int key[CH], dst[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const long long i = b0 + j * 256 + threadIdx.x;
        key[j] = i < n_tot ? D.key[i] : -1;
    }
    // the offsets and ranks of all chunks in flight together: a particle that is not bucketed
    // here reads entry 0 of both (a line the wave shares) and discards it
    int o[CH], r[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const bool mv = key[j] >= 0 && !(key[j] & kStayBit);
        o[j] = D.off[mv ? key[j] : 0];
        r[j] = D.rank[mv ? b0 + j * 256 + threadIdx.x : 0];
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) dst[j] = (key[j] >= 0 && !(key[j] & kStayBit)) ? o[j] + r[j] : -1;
#pragma unroll
    for (int j = 0; j < CH; ++j)
        if (dst[j] >= 0) D.perm[dst[j]] = (int32_t)(b0 + j * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------------------
// Sort by one wave of a short list of distinct ints, ascending.  Bitonic network whose
// comparators all put the smaller value first, so entries past len behave as +infinity and
// are never touched.  a may point to LDS or to global memory; only this wave touches it.
// ---------------------------------------------------------------------------------------
// orders this wave's LDS and global accesses (its lanes run together: no barrier needed)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ void wave_sort(int *a, int len) {
    constexpr int BS = kWave;
    if (len < 2) return;
    const int lane = lane_id();
    int bad = 0;
    for (int i = lane; i + 1 < len; i += BS) bad |= a[i] > a[i + 1];
    if (!__ballot(bad)) return;
    int N = 1;
    while (N < len) N <<= 1;
    for (int k = 2; k <= N; k <<= 1) {
        const int h = k >> 1;
        for (int p = lane; p < N / 2; p += BS) {
            const int i = (p / h) * k + (p % h);
            const int j = i ^ (k - 1);
            if (j < len) {
                int ai = a[i], aj = a[j];
                if (ai > aj) {
                    a[i] = aj;
                    a[j] = ai;
                }
            }
        }
        wave_sync();
        for (int j = h >> 1; j > 0; j >>= 1) {
            for (int p = lane; p < N / 2; p += BS) {
                const int i = (p / j) * 2 * j + (p % j);
                const int q = i + j;
                if (q < len) {
                    int ai = a[i], aq = a[q];
                    if (ai > aq) {
                        a[i] = aq;
                        a[q] = ai;
                    }
                }
            }
            wave_sync();
        }
    }
}



// ---------------------------------------------------------------------------------------
// S6 helpers: records of the gather (k_gather below)
// ---------------------------------------------------------------------------------------
// add phi of a record without copying it (collided particles).  KE: the particles carry an
// internal energy (K > 0); the monatomic instantiations leave it out at compile time, which
// keeps their register counts (and occupancy) those of a kernel without it.
template <bool KE>
__device__ __forceinline__ void add_rec(const Particles &src, int s, double acc[5], double) {
    const double2 *a = reinterpret_cast<const double2 *>(src.rec + s);
    const double2 r1 = a[1], r2 = a[2], r3 = a[3];
    const double u[3] = {r1.y, r2.x, r2.y};
    if constexpr (KE)
        add_phi<double>(acc, r3.x, u, src.e64[s]);
    else
        add_phi<double>(acc, r3.x, u);
}
template <bool KE>
__device__ __forceinline__ void add_rec(const Particles &src, int s, double acc[5], float) {
    const float4 *a = reinterpret_cast<const float4 *>(src.rec32 + s);
    const float4 r0 = a[0], r1 = a[1];
    const float u[3] = {r0.w, r1.x, r1.y};
    if constexpr (KE)
        add_phi<float>(acc, src.m32[s], u, src.e32[s]);
    else
        add_phi<float>(acc, src.m32[s], u);
}

// a whole record in registers, so that several loads can be in flight before the stores
// (scalar arrays: kept in registers, where structs of vectors went to scratch)
struct Rec64 {
    double v[8];  // x0 x1 | x2 u0 | u1 u2 | m id
    double e;     // internal energy variable (K > 0)
};
struct Rec32 {
    float v[9];  // x0 x1 x2 u0 | u1 u2 id.lo id.hi, then m
    float e;
};
template <typename R>
struct RecOf;
template <>
struct RecOf<double> {
    using T = Rec64;
};
template <>
struct RecOf<float> {
    using T = Rec32;
};
template <bool KE>
__device__ __forceinline__ void load_rec(const Particles &src, int s, Rec64 &q) {
    const double2 *a = reinterpret_cast<const double2 *>(src.rec + s);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 t = a[k];
        q.v[2 * k] = t.x;
        q.v[2 * k + 1] = t.y;
    }
    if constexpr (KE) q.e = src.e64[s];
}
template <bool KE>
__device__ __forceinline__ void load_rec(const Particles &src, int s, Rec32 &q) {
    const float4 *a = reinterpret_cast<const float4 *>(src.rec32 + s);
    const float4 t0 = a[0], t1 = a[1];
    q.v[0] = t0.x;
    q.v[1] = t0.y;
    q.v[2] = t0.z;
    q.v[3] = t0.w;
    q.v[4] = t1.x;
    q.v[5] = t1.y;
    q.v[6] = t1.z;
    q.v[7] = t1.w;
    q.v[8] = src.m32[s];
    if constexpr (KE) q.e = src.e32[s];
}
// Staged output: a lane adds phi of its record, puts the record into its slot of the wave's
// LDS stage and writes the small per-particle arrays (cell; FP32: mass) itself; then the wave
// stores the run of staged records with consecutive lanes on consecutive 16-byte chunks, a
// few whole cache lines per instruction instead of a 16-byte piece of 64 lines.
template <bool KE>
__device__ __forceinline__ void stage_rec(const Particles &dst, int o, int c, const Rec64 &q, double acc[5],
                                          uint4 *slot) {
    const double u[3] = {q.v[3], q.v[4], q.v[5]};
    if constexpr (KE)
        add_phi<double>(acc, q.v[6], u, q.e);
    else
        add_phi<double>(acc, q.v[6], u);
    double2 *b = reinterpret_cast<double2 *>(slot);
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = make_double2(q.v[2 * k], q.v[2 * k + 1]);
    dst.cell[o] = c;
    if constexpr (KE) dst.e64[o] = q.e;
}
template <bool KE>
__device__ __forceinline__ void stage_rec(const Particles &dst, int o, int c, const Rec32 &q, double acc[5],
                                          uint4 *slot) {
    const float u[3] = {q.v[3], q.v[4], q.v[5]};
    if constexpr (KE)
        add_phi<float>(acc, q.v[8], u, q.e);
    else
        add_phi<float>(acc, q.v[8], u);
    float4 *b = reinterpret_cast<float4 *>(slot);
    b[0] = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
    b[1] = make_float4(q.v[4], q.v[5], q.v[6], q.v[7]);
    dst.m32[o] = q.v[8];
    dst.cell[o] = c;
    if constexpr (KE) dst.e32[o] = q.e;
}
// a stayer's state at the end of the step: x + u dt (its record holds the start of the step;
// the same arithmetic as the transport's last move of a flight that meets no face)
__device__ __forceinline__ void advance(Rec64 &q, double dt) {
    q.v[0] = q.v[0] + q.v[3] * dt;
    q.v[1] = q.v[1] + q.v[4] * dt;
    q.v[2] = q.v[2] + q.v[5] * dt;
}
__device__ __forceinline__ void advance(Rec32 &q, float dt) {
    q.v[0] = q.v[0] + q.v[3] * dt;
    q.v[1] = q.v[1] + q.v[4] * dt;
    q.v[2] = q.v[2] + q.v[5] * dt;
}

// the wave's n staged records to dst from record o0 on (called by the whole wave; the fences
// order this wave's LDS accesses, which the hardware performs in order)
template <typename R>
__device__ __forceinline__ void stage_out(const uint4 *st, const Particles &dst, int o0, int n) {
    constexpr int CPR = RecChunks<R>::N;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint4 *g = rec_chunks(dst, o0, R(0));
    for (int k = lane_id(); k < n * CPR; k += kWave) st_nt(&g[k], st[k]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// ---------------------------------------------------------------------------------------
// S6: one wave per cell c.  The survivors ending in c are laid out in the next buffer as
//   [movers into c, ascending source index] [stayers of c, in their segment order]
// where stayers (collisionless for the whole step without meeting a face: advanced here by
// u dt) are found by scanning c's own start segments (old particles, then the ones sampled
// this step) and movers (every other survivor, including one that came back to its start
// cell after a wall) come bucketed by k_scatter.  Sums over survivors give P^{n+1}; with the
// collided particles ending in c they give E; then W^{n+1} = W^n + (-sum_f s_f Phi_f + E - S) /
// Omega.  Fixed per-lane assignment and reduction tree: bitwise reproducible.
// ---------------------------------------------------------------------------------------
// The sums follow the output positions: the survivor at position base + l + 64 k is summed by
// lane l, in increasing k, which is the order in which k_heat sums the same particles (so that
// a state imported between steps gets the heat flux the gather would have left, bit for bit).
// After a run of n records is stored from the stage to positions o0.., lane l takes the staged
// record at index (l - (o0 - base)) mod 64.  FP32: the masses are staged beside the records.
__device__ __forceinline__ void stage_mass(float *stm, int k, const Rec64 &) {}
__device__ __forceinline__ void stage_mass(float *stm, int k, const Rec32 &q) { stm[k] = q.v[8]; }
template <typename R>
__device__ __forceinline__ void heat_from_stage(const uint4 *st, const float *stm, int r, int n, double H[9]) {
    const int kk = (lane_id() - r) & (kWave - 1);
    if (kk < n) {
        if constexpr (sizeof(R) == 8) {
            const double2 *a = reinterpret_cast<const double2 *>(st + kk * 4);
            add_heat<true>(a[3].x, a[1].y, a[2].x, a[2].y, H);
        } else {
            const float4 *a = reinterpret_cast<const float4 *>(st + kk * 2);
            add_heat<true>((double)stm[kk], (double)a[0].w, (double)a[1].x, (double)a[1].y, H);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <typename R, int WPB, bool KE, bool SH>
__device__ __forceinline__ void gather_cells(const Dev &D, int buf) {
    constexpr int BS = kWave;
    constexpr int kLds = 256;  // longer source lists are sorted in place in global memory
    constexpr int CPR = RecChunks<R>::N;
    __shared__ int lds_all[WPB][kLds];
    __shared__ uint4 st_all[WPB][kWave * CPR];
    __shared__ float stm_all[WPB][SH ? kWave : 1];  // staged FP32 masses (heat sums)
    // WPB waves per block, one cell each, independent of one another (no block barrier).
    // Blocks go round-robin to the 8 XCDs; give each XCD a contiguous range of cells so
    // that neighbouring cells (whose particles are exchanged) share an L2
    const int G = (int)gridDim.x, bidx = (int)blockIdx.x;
    const int xcd = bidx & 7, q = G >> 3, rr = G & 7;
    const int wave = (int)(threadIdx.x / kWave);
    const int c = (xcd * q + (xcd < rr ? xcd : rr) + (bidx >> 3)) * WPB + wave;
    const int nc = D.nc, nf = D.nf;
    if (c >= nc) return;
    int *lds = lds_all[wave];
    uint4 *st = st_all[wave];
    float *stm = stm_all[wave];
    const int lane = lane_id();
    const Particles src = D.pa[buf], dst = D.pa[buf ^ 1];
    const Scalars *sc = D.sc;
    // every per-cell scalar in one round of independent loads
    const int base = D.off[c], bend = D.off[c + 1];
    const int nmov = (int)(D.cnt64[c] & 0xFFFFFFFFULL);
    const int cb0 = D.off[nc + c], cb1 = D.off[nc + c + 1];
    const long long s00 = D.segoff[buf][c], s01 = D.segoff[buf][c + 1];
    const long long n_old = sc->n_old, n_new = sc->n_new;
    const long long s10 = n_old + D.samoff[c], s11 = n_old + D.samoff[c + 1];
    const int nfc = D.nfc[c];
    // face fluxes of this cell, lane k < 5 owns component k: acc_k = -sum_f s_f Phi_f,k
    const int code = lane < nfc ? D.cface[c * 6 + lane] : 0;
    double facc = 0.0;
    {
        int codes[6];
#pragma unroll
        for (int lf = 0; lf < 6; ++lf) codes[lf] = __shfl(code, lf);
        if (lane < 5) {
            double ph[6];
#pragma unroll
            for (int lf = 0; lf < 6; ++lf) {
                const int cd = codes[lf];
                const int f = (cd > 0 ? cd : -cd) - 1;
                ph[lf] = lf < nfc ? D.Phi[lane * nf + f] : 0.0;
            }
            for (int lf = 0; lf < nfc; ++lf) {
                const double sg = codes[lf] > 0 ? 1.0 : -1.0;
                facc = facc - sg * ph[lf];
            }
        }
    }
    if (nmov == 0 && cb1 == cb0 && s00 == s01 && (n_new == 0 || s10 == s11)) {
        // no particle ends in c and none stays there: the update is -sum_f s_f Phi_f - S, with
        // the particle sums exactly 0 (as the reductions below would give)
        if (lane < 5) {
            const double acc = facc + (0.0 - D.S[lane * nc + c]);
            D.W[lane * nc + c] = D.W[lane * nc + c] + acc / D.vol[c];
            D.P[lane * nc + c] = 0.0;
        }
        if (lane == 0) {
            D.nleft[c] = bend - base;
            D.segoff[buf ^ 1][c] = base;
            if (base != bend) atomicOr(&D.sc->err, kErrCapacity);
        }
        if (SH && lane < 3) D.qh[lane * nc + c] = 0.0;
        return;
    }
    double Pn[5] = {0, 0, 0, 0, 0}, Cn[5] = {0, 0, 0, 0, 0};
    double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const bool shc = SH && D.ip[inst_of(D, c)].pr != 1.0;
    // movers (part 0) and collided (part 1): source lists sorted ascending
    for (int part = 0; part < 2; ++part) {
        const int a0 = part == 0 ? base : cb0;
        const int len = part == 0 ? nmov : cb1 - cb0;
        int *list;
        if (len <= kLds) {
            for (int j = lane; j < len; j += BS) lds[j] = D.perm[a0 + j];
            wave_sync();
            list = lds;
        } else {
            list = D.perm + a0;
        }
        wave_sort(list, len);
        if (part == 0) {
            // two records per lane in flight: both loads before either store
            for (int j0 = 0; j0 < len; j0 += 2 * BS) {
                const int j = j0 + lane;
                const bool ha = j < len, hb = j + BS < len;
                typename RecOf<R>::T A{}, B{};
                if (ha) load_rec<KE>(src, list[j], A);
                if (hb) load_rec<KE>(src, list[j + BS], B);
                if (ha) stage_rec<KE>(dst, a0 + j, c, A, Pn, st + lane * CPR);
                if (SH && ha) stage_mass(stm, lane, A);
                stage_out<R>(st, dst, a0 + j0, min(BS, len - j0));
                if (shc) heat_from_stage<R>(st, stm, (a0 + j0 - base) & 63, min(BS, len - j0), H);
                if (hb) stage_rec<KE>(dst, a0 + j + BS, c, B, Pn, st + lane * CPR);
                if (SH && hb) stage_mass(stm, lane, B);
                stage_out<R>(st, dst, a0 + j0 + BS, max(0, min(BS, len - j0 - BS)));
                if (shc) heat_from_stage<R>(st, stm, (a0 + j0 + BS - base) & 63, max(0, min(BS, len - j0 - BS)), H);
            }
        } else {
#pragma unroll 2
            for (int j = lane; j < len; j += BS) add_rec<KE>(src, list[j], Cn, R(0));
        }
        wave_sync();
    }
    // stayers: own segment of old particles, then own new particles, compacted in order and
    // advanced by u dt (the transport left their records as they were)
    const R dtR = (R)D.is[inst_of(D, c)].dt;
    const unsigned long long below = lane == 0 ? 0ULL : (~0ULL >> (64 - lane));
    int pos = base + nmov;
    for (int seg = 0; seg < 2; ++seg) {
        const long long s0 = seg == 0 ? s00 : s10;
        const long long s1 = seg == 0 ? s01 : (n_new == 0 ? s10 : s11);
        // two runs of 64 per pass: both key loads, then both record loads, then the stores
        for (long long j0 = s0; j0 < s1; j0 += 2 * BS) {
            const long long ja = j0 + lane, jb = j0 + BS + lane;
            const int ka = ja < s1 ? D.key[ja] : -1;
            const int kb = jb < s1 ? D.key[jb] : -1;
            const bool sa = ka >= 0 && (ka & kStayBit) != 0, sb = kb >= 0 && (kb & kStayBit) != 0;
            const unsigned long long ma = __ballot(sa), mb = __ballot(sb);
            typename RecOf<R>::T A{}, B{};
            if (sa) load_rec<KE>(src, (int)ja, A);
            if (sb) load_rec<KE>(src, (int)jb, B);
            if (sa) advance(A, dtR);
            if (sb) advance(B, dtR);
            const int ra = (int)__popcll(ma & below), rb = (int)__popcll(mb & below);
            if (sa) stage_rec<KE>(dst, pos + ra, c, A, Pn, st + ra * CPR);
            if (SH && sa) stage_mass(stm, ra, A);
            stage_out<R>(st, dst, pos, (int)__popcll(ma));
            if (shc) heat_from_stage<R>(st, stm, (pos - base) & 63, (int)__popcll(ma), H);
            pos += (int)__popcll(ma);
            if (sb) stage_rec<KE>(dst, pos + rb, c, B, Pn, st + rb * CPR);
            if (SH && sb) stage_mass(stm, rb, B);
            stage_out<R>(st, dst, pos, (int)__popcll(mb));
            if (shc) heat_from_stage<R>(st, stm, (pos - base) & 63, (int)__popcll(mb), H);
            pos += (int)__popcll(mb);
        }
    }
    double Pk, Ck;
    wave_sum_pc(Pn, Cn, Pk, Ck);
    double Wk = 0.0;
    if (lane < 5) {
        const double E = Pk + Ck;
        const double acc = facc + (E - D.S[lane * nc + c]);
        Wk = D.W[lane * nc + c] + acc / D.vol[c];
        D.W[lane * nc + c] = Wk;
        D.P[lane * nc + c] = Pk;
    }
    if (lane == 0) {
        D.nleft[c] = bend - base;
        D.segoff[buf ^ 1][c] = base;
        if (pos != bend) atomicOr(&D.sc->err, kErrCapacity);
    }
    if constexpr (SH) {
        // sum m c_i |c|^2 = S3_i - 2 sum_j U_j S2_ij - U_i tr S2 + |U|^2 S1_i + 2 U_i (U . S1) - U_i |U|^2 S0
        if (shc) {
#pragma unroll
            for (int k = 0; k < 9; ++k) H[k] = wave_sum(H[k]);
        }
        double Wn[5], Pv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            Wn[k] = __shfl(Wk, k);
            Pv[k] = __shfl(Pk, k);
        }
        if (lane < 3) D.qh[lane * nc + c] = shc ? heat_of(H, Wn, Pv, D.vol[c]) : 0.0;
    }
}

template <typename R, int WPB, bool KE>
__global__ void __launch_bounds__(WPB * 64) k_gather(Dev D, int buf) {
    gather_cells<R, WPB, KE, false>(D, buf);
}
// the gather of a batch with an instance of the Shakhov model (K = 0): also each cell's heat
// flux for the next step
template <typename R, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_gather_sh(Dev D, int buf) {
    gather_cells<R, WPB, false, true>(D, buf);
}

// S6 in a wave-only step with no particle anywhere (none is left, sampled or let in): the
// update W^{n+1} = W^n + (-sum_f s_f Phi_f + E - S) / Omega with E = 0 and S = P = 0, one
// thread per cell, in the arithmetic and order of the gather's cells without particles (so the
// results are those of the full step bit for bit); the bucket offsets are those of empty cells
__global__ void __launch_bounds__(256) k_gks_update(Dev D, int buf) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= D.nc) return;
    const int nc = D.nc, nf = D.nf, nfc = D.nfc[c];
    int codes[6];
#pragma unroll
    for (int lf = 0; lf < 6; ++lf) codes[lf] = lf < nfc ? D.cface[c * 6 + lf] : 0;
    const double vol = D.vol[c];
    // every load before the first store (the stores could alias them as far as the compiler
    // knows, which would otherwise keep one round trip per component)
    double ph[5][6], pv[5], wv[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
#pragma unroll
        for (int lf = 0; lf < 6; ++lf) {
            const int cd = codes[lf];
            const int f = (cd > 0 ? cd : -cd) - 1;
            ph[k][lf] = lf < nfc ? D.Phi[k * nf + f] : 0.0;
        }
        pv[k] = D.P[k * nc + c];
        wv[k] = D.W[k * nc + c];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double facc = 0.0;
        for (int lf = 0; lf < nfc; ++lf) {
            const double sg = codes[lf] > 0 ? 1.0 : -1.0;
            facc = facc - sg * ph[k][lf];
        }
        const double S = pv[k] + 0.0;
        const double acc = facc + (0.0 - S);
        D.W[k * nc + c] = wv[k] + acc / vol;
        D.P[k * nc + c] = 0.0;
    }
    const int base = D.off[c], bend = D.off[c + 1];
    D.nleft[c] = bend - base;
    D.segoff[buf ^ 1][c] = base;
    if (base != bend) atomicOr(&D.sc->err, kErrCapacity);
}

__global__ void __launch_bounds__(256) k_finalize(Dev D, int buf) {
    __shared__ unsigned long long red[2][64];
    Scalars *s = D.sc;
    const long long n_old = s->n_old, n_new = s->n_new, n_inj = s->n_inj;
    const long long n_tot = n_old + n_new + n_inj;
    if (threadIdx.x < 64) {
        red[0][threadIdx.x] = D.spart[threadIdx.x];
        red[1][threadIdx.x] = D.spart[64 + threadIdx.x];
    }
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    // per instance: its particles occupy the buckets of its cell range, its old particles
    // the survivor segments of those cells, its new ones the sampled and entering ranges of
    // its cells and far-field faces; then its own clock advances
    const int nc = D.nc;
    for (int k = threadIdx.x; k < D.n_inst; k += blockDim.x) {
        const InstP &P = D.ip[k];
        InstS &I = D.is[k];
        const long long alive = D.off[P.cell1] - D.off[P.cell0];
        const long long coll = D.off[nc + P.cell1] - D.off[nc + P.cell0];
        const long long old = D.segoff[buf][P.cell1] - D.segoff[buf][P.cell0];
        const long long smp = n_new > 0 ? D.samoff[P.cell1] - D.samoff[P.cell0] : 0;
        const long long inj = (n_inj > 0 && P.ff1 > P.ff0) ? D.injoff[P.ff1] - D.injoff[P.ff0] : 0;
        const long long tot = old + smp + inj;
        I.n_alive = alive;
        I.n_collided = coll;
        I.n_escaped = tot - alive - coll;
        I.n_sampled = smp;
        I.n_injected = inj;
        I.moved_total = I.moved_total + tot;
        I.t = I.t + I.dt;
        I.step = I.step + 1;
        I.dtmin_bits = 0x7FF0000000000000ULL;
    }
    if (threadIdx.x == 0) {
        const long long alive = D.off[nc];
        const long long ended = D.off[2 * nc];
        s->n_cross = red[0][0];
        s->n_wall = red[1][0];
        s->n_collided = (unsigned long long)(ended - alive);
        s->n_escaped = (unsigned long long)(n_tot - ended);
        s->moved_total = s->moved_total + (unsigned long long)n_tot;
        s->n_alive = alive;
        s->n_old = alive;
        D.segoff[buf ^ 1][nc] = (int32_t)alive;
        s->n_new = 0;
        s->n_inj = 0;
        s->t = s->t + s->dt;
        s->step = s->step + 1;
    }
}

// ---------------------------------------------------------------------------------------
// exclusive scan (integers, deterministic): out[i] = sum_{j<i} in[j], out[n] = total
// ---------------------------------------------------------------------------------------
constexpr int kScanBS = 256, kScanPer = 8, kScanTile = kScanBS * kScanPer;

// scan inputs: a plain array, or the bucket sizes (movers / collided in the low word of the
// bucket counter, stayers in the high word)
template <typename T>
struct LoadPlain {
    const T *p;
    __device__ T operator()(long long i) const { return p[i]; }
};
struct LoadBucket {
    const unsigned long long *p;
    __device__ int32_t operator()(long long i) const {
        const unsigned long long v = p[i];
        return (int32_t)(v & 0xFFFFFFFFULL) + (int32_t)(v >> 32);
    }
};

template <typename T>
__device__ T block_exclusive_scan(T v, T *sh, T &total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < kScanBS; s <<= 1) {
        T t = (int)threadIdx.x >= s ? sh[threadIdx.x - s] : T(0);
        __syncthreads();
        sh[threadIdx.x] = sh[threadIdx.x] + t;
        __syncthreads();
    }
    T incl = sh[threadIdx.x];
    total = sh[kScanBS - 1];
    __syncthreads();
    return incl - v;
}

template <typename T, typename L>
__global__ void k_scan_reduce(L in, long long n, T *part) {
    __shared__ T sh[kScanBS];
    const long long base = (long long)blockIdx.x * kScanTile;
    T s = 0;
    for (int q = 0; q < kScanPer; ++q) {
        long long i = base + (long long)threadIdx.x * kScanPer + q;
        if (i < n) s = s + in(i);
    }
    T tot;
    block_exclusive_scan<T>(s, sh, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Each block finds its own offset, the totals of the blocks before it (a few thousand at
// most, read from the L2), so no kernel in between scans the block totals; the last block
// writes the grand total to out[n].  Integer sums: the order does not matter.
template <typename T, typename L>
__global__ void k_scan_apply(L in, long long n, const T *part, T *out) {
    __shared__ T sh[kScanBS];
    T o = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanBS) o = o + part[b];
    T off;
    block_exclusive_scan<T>(o, sh, off);
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanPer;
    T v[kScanPer];
    T s = 0;
    for (int q = 0; q < kScanPer; ++q) {
        long long i = base + q;
        v[q] = i < n ? in(i) : T(0);
        s = s + v[q];
    }
    T tot;
    T ex = block_exclusive_scan<T>(s, sh, tot) + off;
    for (int q = 0; q < kScanPer; ++q) {
        long long i = base + q;
        if (i < n) out[i] = ex;
        ex = ex + v[q];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + tot;
}

template <typename T>
__global__ void k_fill(T *p, long long n, T v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------------------
// Time averaging for steady states (Sec. 2.4(c)): over the steps n > N_avg of an instance,
// Wbar = A / D with A = sum dt^n W^n per cell and D = sum dt^n, and the relative change of
// Wbar in a step, sum_c Omega_c sum_k |Wbar^n - Wbar^{n-1}| / sum_c Omega_c sum_k |Wbar^n|
// (+infinity until two steps are averaged).  k_avg_cells: kAvgBlocks blocks per instance,
// each a contiguous run of its cells, fixed per-thread assignment and reduction tree;
// k_avg_fin: one wave per instance sums its blocks' partials and advances D.  Both run after
// k_finalize (the instance's step counter and dt are those of the step just taken).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_avg_cells(Dev D) {
    __shared__ double red[2][256];
    const int inst = (int)blockIdx.x / kAvgBlocks, j = (int)blockIdx.x % kAvgBlocks;
    const InstS &I = D.is[inst];
    if (I.step <= D.avg_from) return;
    const InstP &P = D.ip[inst];
    const int nc = D.nc, t = (int)threadIdx.x;
    const int n = P.cell1 - P.cell0, chunk = (n + kAvgBlocks - 1) / kAvgBlocks;
    const int c0 = P.cell0 + j * chunk, c1 = min(P.cell1, c0 + chunk);
    const double dt = I.dt, d0 = I.avg_D, d1 = d0 + dt;
    const bool prev = I.avg_n > 0;
    double diff = 0.0, mag = 0.0;
    for (int c = c0 + t; c < c1; c += 256) {
        double dc = 0.0, mc = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double a0 = D.avgA[(long long)k * nc + c];
            const double a1 = a0 + dt * D.W[(long long)k * nc + c];
            D.avgA[(long long)k * nc + c] = a1;
            const double wb1 = a1 / d1;
            mc = mc + fabs(wb1);
            if (prev) dc = dc + fabs(wb1 - a0 / d0);
        }
        const double vol = D.vol[c];
        mag = mag + vol * mc;
        diff = diff + vol * dc;
    }
    red[0][t] = diff;
    red[1][t] = mag;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] = red[0][t] + red[0][t + h];
            red[1][t] = red[1][t] + red[1][t + h];
        }
        __syncthreads();
    }
    if (t < 2) D.avgpart[2 * (long long)blockIdx.x + t] = red[t][0];
}

__global__ void __launch_bounds__(64) k_avg_fin(Dev D) {
    const int inst = (int)blockIdx.x, lane = lane_id();
    InstS &I = D.is[inst];
    if (I.step <= D.avg_from) return;
    double diff = 0.0, mag = 0.0;
    for (int b = lane; b < kAvgBlocks; b += kWave) {
        diff = diff + D.avgpart[2 * ((long long)inst * kAvgBlocks + b)];
        mag = mag + D.avgpart[2 * ((long long)inst * kAvgBlocks + b) + 1];
    }
    diff = wave_sum(diff);
    mag = wave_sum(mag);
    if (lane == 0) {
        I.avg_res = I.avg_n > 0 ? diff / mag : __builtin_inf();
        I.avg_D = I.avg_D + I.dt;
        I.avg_n = I.avg_n + 1;
    }
}

// Wbar = A / D into out, [nc][5]
__global__ void k_avg_out(Dev D, double *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= D.nc) return;
    const double d = D.is[inst_of(D, c)].avg_D;
    for (int k = 0; k < 5; ++k) out[5 * (long long)c + k] = D.avgA[(long long)k * D.nc + c] / d;
}

// field output for ugkwp_moments, [nc][5] in out
__global__ void k_moments(Dev D, int which, double *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= D.nc) return;
    const int nc = D.nc;
    const double vol = D.vol[c];
    double W[5], P[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        W[k] = D.W[k * nc + c];
        P[k] = D.P[k * nc + c] / vol;
    }
    double o[5];
    if (which == 0) {
        for (int k = 0; k < 5; ++k) o[k] = W[k];
    } else if (which == 1) {
        for (int k = 0; k < 5; ++k) o[k] = P[k];
    } else if (which == 2) {
        for (int k = 0; k < 5; ++k) o[k] = W[k] - P[k];
    } else {
        const double rho = W[0];
        o[0] = rho;
        o[1] = W[1] / rho;
        o[2] = W[2] / rho;
        o[3] = W[3] / rho;
        o[4] = temp_k(W, D.K);
    }
    for (int k = 0; k < 5; ++k) out[5 * c + k] = o[k];
}

// exclusive scan of n entries of in into out[0..n]; part: scan_partials_needed(n) entries
template <typename T, typename L>
void scan(L in, long long n, T *out, T *part, hipStream_t s) {
    const int nb = (int)((n + kScanTile - 1) / kScanTile);
    if (nb == 0) {
        k_fill<T><<<1, 1, 0, s>>>(out, 1, T(0));
        return;
    }
    k_scan_reduce<T, L><<<nb, kScanBS, 0, s>>>(in, n, part);
    k_scan_apply<T, L><<<nb, kScanBS, 0, s>>>(in, n, part, out);
}

}  // namespace

long long scan_partials_needed(long long n) { return (n + kScanTile - 1) / kScanTile + 1; }


void launch_fill_i32(int32_t *p, long long n, int32_t v, hipStream_t s) {
    if (n > 0) k_fill<int32_t><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}
void launch_fill_f64(double *p, long long n, double v, hipStream_t s) {
    if (n > 0) k_fill<double><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

namespace {
// entries of one wall-queue segment for a transport grid of g blocks of `per` particles;
// kWallSeg segments take at most cap + kWallSlack entries
long long wall_qseg(long long g, long long per) { return (g + kWallSeg - 1) / kWallSeg * per; }

template <typename R, bool MULTI, int ILP>
long long launch_stream_i(const Dev &D, int buf, int bs, hipStream_t s) {
    // ILP particles per thread over the capacity; blocks past the live particles exit at once
    const long long per = (long long)bs * ILP;
    const unsigned g = (unsigned)((D.cap + per - 1) / per);
    const long long qseg = wall_qseg(g, per);
    if (bs == 128)
        k_stream<R, 128, MULTI, ILP><<<g, 128, 0, s>>>(D, buf, qseg);
    else if (bs == 512)
        k_stream<R, 512, MULTI, ILP><<<g, 512, 0, s>>>(D, buf, qseg);
    else
        k_stream<R, 256, MULTI, ILP><<<g, 256, 0, s>>>(D, buf, qseg);
    return qseg;
}

template <typename R, bool MULTI>
long long launch_stream_t(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s) {
    if (cfg.stream_ilp == 2) return launch_stream_i<R, MULTI, 2>(D, buf, cfg.stream_bs, s);
    return launch_stream_i<R, MULTI, 1>(D, buf, cfg.stream_bs, s);
}

// returns the wall-queue segment length the transport grid used
template <typename R>
long long launch_stream(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s) {
    if (D.n_inst > 1) return launch_stream_t<R, true>(D, buf, cfg, s);
    return launch_stream_t<R, false>(D, buf, cfg, s);
}

template <typename R>
void launch_stream_wall(const Dev &D, int buf, long long qseg, hipStream_t s) {
    // 16 blocks per queue segment, each segment's length known only on the device
    const unsigned g = 16 * kWallSeg;
    if (D.n_inst > 1 && D.K > 0)
        k_stream_wall<R, true, true><<<g, 256, 0, s>>>(D, buf, qseg);
    else if (D.n_inst > 1)
        k_stream_wall<R, true, false><<<g, 256, 0, s>>>(D, buf, qseg);
    else if (D.K > 0)
        k_stream_wall<R, false, true><<<g, 256, 0, s>>>(D, buf, qseg);
    else
        k_stream_wall<R, false, false><<<g, 256, 0, s>>>(D, buf, qseg);
}

template <typename R, bool KE, int G>
void launch_sample_g(const Dev &D, int buf, int w, hipStream_t s) {
    const unsigned g = (unsigned)((D.nc + w * G - 1) / (w * G));
    if (w == 1)
        k_sample<R, 1, KE, G><<<g, 64, 0, s>>>(D, buf);
    else if (w == 2)
        k_sample<R, 2, KE, G><<<g, 128, 0, s>>>(D, buf);
    else if (w == 8)
        k_sample<R, 8, KE, G><<<g, 512, 0, s>>>(D, buf);
    else
        k_sample<R, 4, KE, G><<<g, 256, 0, s>>>(D, buf);
}

// the cells of at most 64 new particles, then those with more
template <typename R, bool KE>
void launch_sample_k(const Dev &D, int buf, int w, hipStream_t s) {
    if (D.nc >= kSampleCellsMin)
        launch_sample_g<R, KE, kSampleCells>(D, buf, w, s);
    else
        launch_sample_g<R, KE, 1>(D, buf, w, s);
    // at most a wave per cell; a grid of a few thousand waves takes any list in turns
    const unsigned gb = (unsigned)std::min<long long>((D.nc + 7) / 8, 2048);
    k_sample_big<R, KE><<<gb, 512, 0, s>>>(D, buf);
}

template <typename R>
void launch_sample(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s) {
    const int w = cfg.sample_wpb, nc = D.nc;
    if (D.K > 0)
        launch_sample_k<R, true>(D, buf, w, s);
    else
        launch_sample_k<R, false>(D, buf, w, s);
    if (D.gp_any) {
        const unsigned g4 = (unsigned)((nc + 3) / 4);
        if (D.K > 0)
            k_sample_gp<R, true><<<g4, 256, 0, s>>>(D, buf);
        else
            k_sample_gp<R, false><<<g4, 256, 0, s>>>(D, buf);
    }
}

template <typename R>
void launch_flux(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s) {
    const int bs = cfg.flux_bs, nf = D.nf;
    const unsigned g = (unsigned)((nf + bs - 1) / bs);
    if (D.recon_any) {
        // second order: gradients (one thread per cell), then the faces of reconstructing
        // instances; the first-order kernel takes the others
        k_grad<<<(unsigned)((D.nc + 127) / 128), 128, 0, s>>>(D);
        if (bs == 64)
            k_flux2<R, 64><<<g, 64, 0, s>>>(D);
        else if (bs == 256)
            k_flux2<R, 256><<<g, 256, 0, s>>>(D);
        else
            k_flux2<R, 128><<<g, 128, 0, s>>>(D);
        if (D.recon_all) return;
    }
    if (bs == 64)
        k_flux<R, 64><<<g, 64, 0, s>>>(D);
    else if (bs == 256)
        k_flux<R, 256><<<g, 256, 0, s>>>(D);
    else
        k_flux<R, 128><<<g, 128, 0, s>>>(D);
}
}  // namespace

void launch_heat(const Dev &D, int buf, hipStream_t s) {
    if (!D.sh_any) return;
    if (D.prec == 1)
        k_heat<float><<<(unsigned)((D.nc + 3) / 4), 256, 0, s>>>(D, buf);
    else
        k_heat<double><<<(unsigned)((D.nc + 3) / 4), 256, 0, s>>>(D, buf);
}

bool launch_cfg_valid(const LaunchCfg &c) {
    const bool sb = (c.stream_bs == 128 || c.stream_bs == 256 || c.stream_bs == 512) &&
                    (c.stream_ilp == 1 || c.stream_ilp == 2);
    const bool sw = c.sample_wpb == 1 || c.sample_wpb == 2 || c.sample_wpb == 4 || c.sample_wpb == 8;
    const bool fb = c.flux_bs == 64 || c.flux_bs == 128 || c.flux_bs == 256;
    return sb && sw && fb;
}

void launch_step(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s, Prof *pr) {
    const int nc = D.nc, nf = D.nf;
    const unsigned gc = (unsigned)((nc + 255) / 256);
    Prof none;
    if (!pr) pr = &none;
    pr->begin(kSlotPrim);
    k_prim_dt<<<gc, 256, 0, s>>>(D);
    pr->end(kSlotPrim);
    pr->begin(kSlotCellPrep);
    k_cell_prep<<<gc, 256, 0, s>>>(D);
    pr->end(kSlotCellPrep);
    pr->begin(kSlotScan);
    scan<long long>(LoadPlain<long long>{D.nsam}, nc, D.samoff, D.scan64, s);
    if (D.nff > 0) {
        k_inject_count<<<(unsigned)((D.nff + 255) / 256), 256, 0, s>>>(D);
        scan<long long>(LoadPlain<long long>{D.ninj}, D.nff, D.injoff, D.scan64, s);
    }
    k_sample_setup<<<1, 1, 0, s>>>(D);
    pr->end(kSlotScan);
    const bool f32 = D.prec == 1;
    pr->begin(kSlotFlux);
    if (nf > 0) {
        if (f32)
            launch_flux<float>(D, buf, cfg, s);
        else
            launch_flux<double>(D, buf, cfg, s);
    }
    pr->end(kSlotFlux);
    pr->begin(kSlotSample);
    if (f32)
        launch_sample<float>(D, buf, cfg, s);
    else
        launch_sample<double>(D, buf, cfg, s);
    if (D.nff > 0) {
        if (f32)
            k_inject<float><<<(unsigned)D.nff, 64, 0, s>>>(D, buf);
        else
            k_inject<double><<<(unsigned)D.nff, 64, 0, s>>>(D, buf);
    }
    pr->end(kSlotSample);
    pr->begin(kSlotStream);
    const long long qseg = f32 ? launch_stream<float>(D, buf, cfg, s) : launch_stream<double>(D, buf, cfg, s);
    pr->end(kSlotStream);
    pr->begin(kSlotStreamWall);
    if (D.any_diffuse) {
        if (f32)
            launch_stream_wall<float>(D, buf, qseg, s);
        else
            launch_stream_wall<double>(D, buf, qseg, s);
    }
    pr->end(kSlotStreamWall);
    pr->begin(kSlotCount);
    if (D.count_ch == 4)
        k_count<4><<<(unsigned)((D.cap + 256 * 4 - 1) / (256 * 4)), 256, 0, s>>>(D);
    else
        k_count<8><<<(unsigned)((D.cap + 256 * 8 - 1) / (256 * 8)), 256, 0, s>>>(D);
    pr->end(kSlotCount);
    pr->begin(kSlotScan2);
    scan<int32_t>(LoadBucket{D.cnt64}, 2LL * nc, D.off, D.scan32, s);
    pr->end(kSlotScan2);
    pr->begin(kSlotScatter);
    k_scatter<<<(unsigned)((D.cap + 256 * kScatterChunks - 1) / (256 * kScatterChunks)), 256, 0, s>>>(D);
    pr->end(kSlotScatter);
    pr->begin(kSlotGather);
    {
        constexpr int WPB = kGatherWaves;
        const unsigned g = (unsigned)((nc + WPB - 1) / WPB);
        if (D.sh_any && f32)
            k_gather_sh<float, WPB><<<g, WPB * 64, 0, s>>>(D, buf);
        else if (D.sh_any)
            k_gather_sh<double, WPB><<<g, WPB * 64, 0, s>>>(D, buf);
        else if (f32 && D.K > 0)
            k_gather<float, WPB, true><<<g, WPB * 64, 0, s>>>(D, buf);
        else if (f32)
            k_gather<float, WPB, false><<<g, WPB * 64, 0, s>>>(D, buf);
        else if (D.K > 0)
            k_gather<double, WPB, true><<<g, WPB * 64, 0, s>>>(D, buf);
        else
            k_gather<double, WPB, false><<<g, WPB * 64, 0, s>>>(D, buf);
    }
    pr->end(kSlotGather);
    pr->begin(kSlotFinal);
    k_finalize<<<1, 256, 0, s>>>(D, buf);
    if (D.avg_from >= 0) {
        k_avg_cells<<<(unsigned)(D.n_inst * kAvgBlocks), 256, 0, s>>>(D);
        k_avg_fin<<<(unsigned)D.n_inst, 64, 0, s>>>(D);
    }
    pr->end(kSlotFinal);
}

// A wave-only step when no particle exists: no particle is sampled or let in (e = 0 in the
// wave-only phase), so the particle kernels would find nothing to do; the bucket counts (zeroed
// by k_prim_dt) are still scanned so that the offsets are those of empty cells.
void launch_step_wave_only(const Dev &D, int buf, const LaunchCfg &cfg, hipStream_t s, Prof *pr) {
    const int nc = D.nc, nf = D.nf;
    const unsigned gc = (unsigned)((nc + 255) / 256);
    Prof none;
    if (!pr) pr = &none;
    pr->begin(kSlotPrim);
    k_prim_dt<<<gc, 256, 0, s>>>(D);
    pr->end(kSlotPrim);
    pr->begin(kSlotCellPrep);
    k_cell_prep<<<gc, 256, 0, s>>>(D);
    pr->end(kSlotCellPrep);
    pr->begin(kSlotScan);
    scan<long long>(LoadPlain<long long>{D.nsam}, nc, D.samoff, D.scan64, s);
    if (D.nff > 0) {
        k_inject_count<<<(unsigned)((D.nff + 255) / 256), 256, 0, s>>>(D);
        scan<long long>(LoadPlain<long long>{D.ninj}, D.nff, D.injoff, D.scan64, s);
    }
    k_sample_setup<<<1, 1, 0, s>>>(D);
    pr->end(kSlotScan);
    pr->begin(kSlotFlux);
    if (nf > 0) {
        if (D.prec == 1)
            launch_flux<float>(D, buf, cfg, s);
        else
            launch_flux<double>(D, buf, cfg, s);
    }
    pr->end(kSlotFlux);
    pr->begin(kSlotScan2);
    scan<int32_t>(LoadBucket{D.cnt64}, 2LL * nc, D.off, D.scan32, s);
    pr->end(kSlotScan2);
    pr->begin(kSlotGather);
    k_gks_update<<<gc, 256, 0, s>>>(D, buf);
    pr->end(kSlotGather);
    pr->begin(kSlotFinal);
    k_finalize<<<1, 256, 0, s>>>(D, buf);
    if (D.avg_from >= 0) {
        k_avg_cells<<<(unsigned)(D.n_inst * kAvgBlocks), 256, 0, s>>>(D);
        k_avg_fin<<<(unsigned)D.n_inst, 64, 0, s>>>(D);
    }
    pr->end(kSlotFinal);
}

void launch_avg_out(const Dev &D, double *out, hipStream_t s) {
    k_avg_out<<<(unsigned)((D.nc + 255) / 256), 256, 0, s>>>(D, out);
}

void launch_moments(const Dev &D, int which, double *out, hipStream_t s) {
    k_moments<<<(unsigned)((D.nc + 255) / 256), 256, 0, s>>>(D, which, out);
}

}  // namespace ugkwp
