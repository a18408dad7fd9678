// Device-side data views and numerical building blocks of the cut-cell split step.
//
// Gas model (Sec. 2.1): Q = (rho, rho u, rho v, E), p = (gamma-1)(E - |m|^2 / (2 rho)).
// Numerical flux (Sec. 2.3.5 end): MUSCL-Hancock with a van Leer limiter on the
// conserved variables, HLLC with Davis wave-speed estimates.
// Geometry (Sec. 2.1-2.2): vertex classes, face solid intervals, cut-cell volume
// fractions of a convex polygon on a uniform Cartesian grid.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc {

enum { FLUID = 0, SOLID = 1 };

struct Grid {
    int nx, ny;
    int bc[4];  // W, E, S, N: 0 zero-gradient, 1 reflective
    double x_lo, y_lo, hx, hy;
    double gamma;
    double alpha_min;  // small-cell threshold: cut cells with a smaller volume fraction are solid
};

// Global-memory view of a pointer.  Pointers that reach a kernel through an argument block
// in device memory have no provable address space, so the compiler emits flat accesses for
// them, and a flat access counts against the LDS completion counter as well: every wait for
// LDS data would also wait for the loads in flight.  The streaming kernels access the state
// through these views.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* to_global(T* p) { return (gmem<T>*)p; }

// Cell index box, half-open [i0, i1) x [j0, j1).
struct Box {
    int i0, i1, j0, j1;
    __host__ __device__ int w() const { return i1 - i0; }
    __host__ __device__ int h() const { return j1 - j0; }
    __host__ __device__ bool has(int i, int j) const { return i >= i0 && i < i1 && j >= j0 && j < j1; }
};

// Posed convex polygon of one level (device copy) and quick-test data.
struct Poly {
    const double* v;  // 2*m, counter-clockwise
    int m;
    double xmin, xmax, ymin, ymax;  // bounding box
    double cx, cy, rin2, rout2;     // certificate disc radii about (cx, cy); rin2 < 0: unused
    // Vertices of least and greatest y (ib, it) and x (il, ir).  Counter-clockwise, y does
    // not decrease from ib to it and x does not decrease from il to ir (the other way round
    // on the remaining chain), so the edges meeting a line or a strip are found by bisection.
    int ib, it, il, ir;
};

// One level: vertex classes, face solid intervals (lo, hi) measured from the face's
// low-index vertex, volume fractions.
struct Level {
    int8_t* vcls;  // (ny+1)*(nx+1)
    double2* fx;   // ny*(nx+1): x-face (i, j) from vertex (i, j) to (i, j+1)
    double2* fy;   // (ny+1)*nx: y-face (i, j) from vertex (i, j) to (i+1, j)
    double* alpha; // ny*nx
    Poly poly;
    // several bodies (np >= 2; else 0 and null): their posed polygons, and the body that
    // cuts each cut cell of the level (-1 elsewhere)
    const Poly* parts;
    int np;
    int8_t* cbody;
};
constexpr int MAX_BODIES = 4;

__device__ __forceinline__ double vx_of(const Grid& g, int i) { return g.x_lo + (double)i * g.hx; }
__device__ __forceinline__ double vy_of(const Grid& g, int j) { return g.y_lo + (double)j * g.hy; }

__device__ __forceinline__ double interval_beta(double2 iv) { return iv.y > iv.x ? 1.0 - (iv.y - iv.x) : 1.0; }

__device__ __forceinline__ double beta_x(const Grid& g, const Level& L, int i, int j) {
    return interval_beta(L.fx[(size_t)j * (g.nx + 1) + i]);
}
__device__ __forceinline__ double beta_y(const Grid& g, const Level& L, int i, int j) {
    return interval_beta(L.fy[(size_t)j * g.nx + i]);
}
__device__ __forceinline__ double alpha_of(const Grid& g, const Level& L, int i, int j) {
    return L.alpha[(size_t)j * g.nx + i];
}

__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double px, double py) {
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

// ------------------------------------------------------------------------------ gas model
// Division and square root.  FP64 (the reference arithmetic, also used for every cut-cell
// quantity in both precision modes) uses correctly rounded IEEE operations in the written
// order.  The FP32 state mode uses the hardware reciprocal and square root (about 1 ulp):
// an IEEE FP32 division expands to ~10 instructions and these sweeps are bound by vector
// ALU issue, not by memory.
template <typename T>
__device__ __forceinline__ T qdiv(T a, T b) {
    return a / b;
}
template <>
__device__ __forceinline__ float qdiv<float>(float a, float b) {
    return a * __builtin_amdgcn_rcpf(b);
}
template <typename T>
__device__ __forceinline__ T qsqrt(T a) {
    return sqrt(a);
}
template <>
__device__ __forceinline__ float qsqrt<float>(float a) {
    return __builtin_amdgcn_sqrtf(a);
}

template <typename T>
__device__ __forceinline__ T pressure(const T q[4], T g) {
    return (g - T(1)) * (q[3] - qdiv(T(0.5) * (q[1] * q[1] + q[2] * q[2]), q[0]));
}

template <typename T, int D>
__device__ __forceinline__ void euler_flux(const T q[4], T g, T f[4]) {
    constexpr int n = 1 + D, t = 2 - D;
    T p = pressure(q, g);
    T un = qdiv(q[n], q[0]);
    f[0] = q[n];
    f[n] = q[n] * un + p;
    f[t] = q[t] * un;
    f[3] = un * (q[3] + p);
}

// ------------------------------------------------------------- FP32 state arithmetic
// The FP32 state mode evaluates the same formulas with one hardware reciprocal of the
// density per state (velocity, pressure, sound speed and flux all reuse it) and fused
// multiply-adds; the FP64 path below keeps every division and the written order.
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// (gamma - 1) (E - |m|^2 / (2 rho)), with ir = 1 / rho
__device__ __forceinline__ float pressure32(const float q[4], float ir, float gm1) {
    float ke = __builtin_fmaf(q[1], q[1], q[2] * q[2]) * (0.5f * ir);
    return gm1 * (q[3] - ke);
}

template <int D>
__device__ __forceinline__ void euler_flux32(const float q[4], float un, float p, float f[4]) {
    constexpr int n = 1 + D, t = 2 - D;
    f[0] = q[n];
    f[n] = __builtin_fmaf(q[n], un, p);
    f[t] = q[t] * un;
    f[3] = un * (q[3] + p);
}

template <int D>
__device__ __forceinline__ void hllc32(const float ql[4], const float qr[4], float g, float f[4]) {
    constexpr int n = 1 + D, t = 2 - D;
    float gm1 = g - 1.0f;
    float rl = ql[0], rr = qr[0];
    float irl = rcp32(rl), irr = rcp32(rr);
    float ul = ql[n] * irl, ur = qr[n] * irr;
    float pl = pressure32(ql, irl, gm1), pr = pressure32(qr, irr, gm1);
    float al = __builtin_amdgcn_sqrtf(g * pl * irl), ar = __builtin_amdgcn_sqrtf(g * pr * irr);
    float sl = fminf(ul - al, ur - ar);
    float sr = fmaxf(ul + al, ur + ar);
    float dl = sl - ul, dr = sr - ur;
    float ml = rl * dl, mr = rr * dr;  // mass fluxes relative to the outer waves
    float ss = __builtin_fmaf(ml, ul, __builtin_fmaf(-mr, ur, pr - pl)) * rcp32(ml - mr);
    int kc = 0.0f <= sl ? 0 : (0.0f <= ss ? 1 : (0.0f <= sr ? 2 : 3));
    bool left = kc <= 1;
    float q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = left ? ql[k] : qr[k];
    float irk = left ? irl : irr, uk = left ? ul : ur, pk = left ? pl : pr, sk = left ? sl : sr;
    float mk = left ? ml : mr;
    float fk[4];
    euler_flux32<D>(q, uk, pk, fk);
    if (kc == 0 || kc == 3) {
#pragma unroll
        for (int k = 0; k < 4; k++) f[k] = fk[k];
        return;
    }
    // star state on the upwind side: c = rho_K (S_K - u_K) / (S_K - S*); the energy's
    // p_K / (rho_K (S_K - u_K)) term times c is p_K / (S_K - S*), so one reciprocal serves
    float rs = rcp32(sk - ss);
    float c = mk * rs;
    float ds = ss - uk;
    float us[4];
    us[0] = c;
    us[n] = c * ss;
    us[t] = c * (q[t] * irk);
    us[3] = __builtin_fmaf(c, __builtin_fmaf(ds, ss, q[3] * irk), ds * pk * rs);
#pragma unroll
    for (int k = 0; k < 4; k++) f[k] = __builtin_fmaf(sk, us[k] - q[k], fk[k]);
}

__device__ __forceinline__ float vanleer32(float a, float b) {
    float ab = a * b;
    return ab > 0.0f ? (ab + ab) * rcp32(a + b) : 0.0f;
}

template <int D>
__device__ __forceinline__ void muscl32(const float qm[4], const float q[4], const float qp[4], bool slope_ok,
                                        float lam, float g, float el[4], float er[4]) {
    constexpr int n = 1 + D;
    float gm1 = g - 1.0f;
    float ql[4], qr[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float d = slope_ok ? vanleer32(q[k] - qm[k], qp[k] - q[k]) : 0.0f;
        ql[k] = __builtin_fmaf(-0.5f, d, q[k]);
        qr[k] = __builtin_fmaf(0.5f, d, q[k]);
    }
    float irl = rcp32(ql[0]), irr = rcp32(qr[0]);
    float pl = pressure32(ql, irl, gm1), pr = pressure32(qr, irr, gm1);
    bool ok = ql[0] > 0.0f && pl > 0.0f && qr[0] > 0.0f && pr > 0.0f;
    if (ok) {
        float fl[4], fr[4];
        euler_flux32<D>(ql, ql[n] * irl, pl, fl);
        euler_flux32<D>(qr, qr[n] * irr, pr, fr);
        float hl = 0.5f * lam;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            float c = hl * (fl[k] - fr[k]);
            el[k] = ql[k] + c;
            er[k] = qr[k] + c;
        }
        // p > 0 with rho > 0 is 2 rho E > |m|^2 (no reciprocal needed for the test)
        ok = el[0] > 0.0f && er[0] > 0.0f &&
             __builtin_fmaf(el[1], el[1], el[2] * el[2]) < 2.0f * el[0] * el[3] &&
             __builtin_fmaf(er[1], er[1], er[2] * er[2]) < 2.0f * er[0] * er[3];
    }
    if (!ok) {
#pragma unroll
        for (int k = 0; k < 4; k++) el[k] = er[k] = q[k];
    }
}

// Signal speeds |u|+a and |v|+a of a regular cell's FP32 state as bit patterns of
// non-negative floats (they order like the values, as unsigned integers; NaN maps to the
// quiet NaN above infinity), and the conversion of such a pattern to the FP64 one of the
// same value.  Float to double is exact and monotone, so the maximum of converted patterns
// is the converted maximum.
__device__ __forceinline__ void speed_bits32(const float u[4], float g, unsigned& bx, unsigned& by) {
    float ir = rcp32(u[0]);
    float uu = u[1] * ir, vv = u[2] * ir;
    float c = __builtin_amdgcn_sqrtf(g * pressure32(u, ir, g - 1.0f) * ir);
    float sx = fabsf(uu) + c, sy = fabsf(vv) + c;
    bx = sx != sx ? 0x7fc00000u : __float_as_uint(sx);
    by = sy != sy ? 0x7fc00000u : __float_as_uint(sy);
}
__device__ __forceinline__ unsigned long long bits32_to_64(unsigned b) {
    return b > 0x7f800000u ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong((double)__uint_as_float(b));
}

// Signal speeds |u|+a and |v|+a of a stored state u (conserved per cell volume) with volume
// fraction alpha, as bit patterns of non-negative doubles (they order like the values; NaN
// maps above infinity); 0 for cells without gas.  A regular cell (alpha 1) is evaluated in
// the state's precision, a cut cell in FP64 from U / alpha.  Every time-step reduction uses
// this one rule, so their maxima agree bit for bit.
template <typename R>
__device__ __forceinline__ void speed_bits(const R u[4], double alpha, double gam, unsigned long long& bx,
                                           unsigned long long& by) {
    bx = by = 0ull;
    if (!(alpha > 0.0) || !((double)u[0] > 0.0)) return;
    double sx, sy;
    if (alpha == 1.0) {
        R g = (R)gam;
        if constexpr (sizeof(R) == 4) {
            unsigned x, y;
            speed_bits32(u, g, x, y);
            bx = bits32_to_64(x);
            by = bits32_to_64(y);
            return;
        } else {
            R uu = qdiv(u[1], u[0]), vv = qdiv(u[2], u[0]);
            R c = qsqrt(qdiv(g * pressure(u, g), u[0]));
            sx = (double)(fabs(uu) + c);
            sy = (double)(fabs(vv) + c);
        }
    } else {
        double q[4];
#pragma unroll
        for (int m = 0; m < 4; m++) q[m] = (double)u[m] / alpha;
        double uu = q[1] / q[0], vv = q[2] / q[0];
        double c = sqrt(gam * pressure(q, gam) / q[0]);
        sx = fabs(uu) + c;
        sy = fabs(vv) + c;
    }
    bx = __double_as_longlong(sx);
    by = __double_as_longlong(sy);
    if (sx != sx) bx = 0x7ff8000000000000ull;
    if (sy != sy) by = 0x7ff8000000000000ull;
}

// HLLC flux with Davis wave-speed estimates.  The two star-region cases share one code
// path on the upwind side's values (same operations as writing them out per side).
template <typename T, int D>
__device__ __forceinline__ void hllc(const T ql[4], const T qr[4], T g, T f[4]) {
    if constexpr (sizeof(T) == 4) {
        hllc32<D>(ql, qr, g, f);
        return;
    }
    constexpr int n = 1 + D, t = 2 - D;
    T rl = ql[0], rr = qr[0];
    T ul = qdiv(ql[n], rl), ur = qdiv(qr[n], rr);
    T pl = pressure(ql, g), pr = pressure(qr, g);
    T al = qsqrt(qdiv(g * pl, rl)), ar = qsqrt(qdiv(g * pr, rr));
    T sl = fmin(ul - al, ur - ar);
    T sr = fmax(ul + al, ur + ar);
    T ss = qdiv(pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur), rl * (sl - ul) - rr * (sr - ur));
    // 0: F_L (0 <= S_L); 1: star L (0 <= S*); 2: star R (0 <= S_R); 3: F_R
    int kc = T(0) <= sl ? 0 : (T(0) <= ss ? 1 : (T(0) <= sr ? 2 : 3));
    bool left = kc <= 1;
    T q[4];  // upwind state, selected by value (a selected pointer would force both arrays to memory)
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = left ? ql[k] : qr[k];
    if (kc == 0 || kc == 3) {
        euler_flux<T, D>(q, g, f);  // supersonic: the upwind state's flux
        return;
    }
    // star region on the upwind side K: F_K + S_K (U*_K - U_K)
    T rk = left ? rl : rr, uk = left ? ul : ur, pk = left ? pl : pr, sk = left ? sl : sr;
    T fk[4];
    euler_flux<T, D>(q, g, fk);
    T c = qdiv(rk * (sk - uk), sk - ss);
    T us[4];
    us[0] = c;
    us[n] = c * ss;
    us[t] = c * qdiv(q[t], rk);
    us[3] = c * (qdiv(q[3], rk) + (ss - uk) * (ss + qdiv(pk, rk * (sk - uk))));
#pragma unroll
    for (int k = 0; k < 4; k++) f[k] = fk[k] + sk * (us[k] - q[k]);
}

template <typename T>
__device__ __forceinline__ T vanleer(T a, T b) {
    return a * b > T(0) ? qdiv(T(2) * a * b, a + b) : T(0);
}

template <typename T>
__device__ __forceinline__ bool admissible(const T q[4], T g) {
    if (!(q[0] > T(0))) return false;
    return pressure(q, g) > T(0);
}

// MUSCL-Hancock reconstruction and half-step evolution of one cell; el/er are the
// evolved states at the cell's low and high faces.  Positivity fallback: drop the slope.
template <typename T, int D>
__device__ __forceinline__ void muscl(const T qm[4], const T q[4], const T qp[4], bool slope_ok, T lam, T g,
                                      T el[4], T er[4]) {
    if constexpr (sizeof(T) == 4) {
        muscl32<D>(qm, q, qp, slope_ok, lam, g, el, er);
        return;
    }
    T dl[4];
#pragma unroll
    for (int k = 0; k < 4; k++) dl[k] = slope_ok ? vanleer(q[k] - qm[k], qp[k] - q[k]) : T(0);
    bool ok = true;
    {
        T ql[4], qr[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            ql[k] = q[k] - T(0.5) * dl[k];
            qr[k] = q[k] + T(0.5) * dl[k];
        }
        ok = admissible(ql, g) && admissible(qr, g);
        if (ok) {
            T fl[4], fr[4];
            euler_flux<T, D>(ql, g, fl);
            euler_flux<T, D>(qr, g, fr);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                T c = T(0.5) * lam * (fl[k] - fr[k]);
                el[k] = ql[k] + c;
                er[k] = qr[k] + c;
            }
            ok = admissible(el, g) && admissible(er, g);
        }
    }
    if (!ok) {
        // flat profile: the half-step evolution of a constant state is the state itself
#pragma unroll
        for (int k = 0; k < 4; k++) el[k] = er[k] = q[k];
    }
}

}  // namespace cc
