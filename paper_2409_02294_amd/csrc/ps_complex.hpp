// Complex arithmetic and small in-register DFTs for the gfx950 kernels.
//
// Sign convention: DIR = -1 is the forward transform, exp(-2 pi i jk / n);
// DIR = +1 the inverse, exp(+2 pi i jk / n), neither normalised.  The
// constants are written in double precision and rounded once to T.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace ps {

template <typename T> struct cx_of;
template <> struct cx_of<float> { using type = float2; };
template <> struct cx_of<double> { using type = double2; };
template <typename T> using cx = typename cx_of<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b)
{
    return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
template <typename V, typename T> __device__ __forceinline__ V cscale(V a, T s) { return V{a.x * s, a.y * s}; }
// a * w for w = DIR ? conj : plain, used to apply a forward-sign table entry in either direction
template <int DIR, typename V> __device__ __forceinline__ V ctw(V a, V w)
{
    if constexpr (DIR < 0) return cmul(a, w);
    else return cmulc(a, w);
}
// a * (DIR i)
template <int DIR, typename V> __device__ __forceinline__ V crot(V a)
{
    if constexpr (DIR < 0) return V{a.y, -a.x};
    else return V{-a.y, a.x};
}

// a * exp(DIR * 2 pi i * M / 16), M in [0, 16)
template <int DIR, int M, typename V> __device__ __forceinline__ V w16(V a)
{
    using T = decltype(a.x);
    constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double H = 0.70710678118654752440;   // sqrt(1/2)
    constexpr int m = M & 15;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return crot<DIR>(a);
    else if constexpr (m == 8) return V{-a.x, -a.y};
    else if constexpr (m == 12) return crot<-DIR>(a);
    else if constexpr (m == 2 || m == 6 || m == 10 || m == 14) {
        // exp(DIR i pi m/8) with m/2 odd: (+-H, +-H)
        constexpr double cr = (m == 2 || m == 14) ? H : -H;
        constexpr double ci0 = (m == 2 || m == 6) ? H : -H;
        constexpr double ci = DIR < 0 ? -ci0 : ci0;
        const T c = T(cr), s = T(ci);
        return V{a.x * c - a.y * s, a.x * s + a.y * c};
    } else {
        // odd m: cos / sin of m pi / 8
        constexpr int q = m;  // 1,3,5,7,9,11,13,15
        constexpr double cr = (q == 1 || q == 15) ? C1 : (q == 3 || q == 13) ? S1 : (q == 5 || q == 11) ? -S1 : -C1;
        constexpr double si0 = (q == 1 || q == 7) ? S1 : (q == 3 || q == 5) ? C1 : (q == 9 || q == 15) ? -S1 : -C1;
        constexpr double ci = DIR < 0 ? -si0 : si0;
        const T c = T(cr), s = T(ci);
        return V{a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// ---------------------------------------------------------------------------
// In-register DFTs, natural order in and out: v[k] <- sum_j v[j] w_R^(jk).
// ---------------------------------------------------------------------------

template <int DIR, typename V> __device__ __forceinline__ void dft2(V* v)
{
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int DIR, typename V> __device__ __forceinline__ void dft4v(V& a0, V& a1, V& a2, V& a3)
{
    V t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = crot<DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <int DIR, typename V> __device__ __forceinline__ void dft4(V* v) { dft4v<DIR>(v[0], v[1], v[2], v[3]); }

template <int DIR, typename V> __device__ __forceinline__ void dft3(V* v)
{
    using T = decltype(v[0].x);
    constexpr double S3 = 0.86602540378443864676;  // sqrt(3)/2
    V a0 = v[0], a1 = v[1], a2 = v[2];
    V t = cadd(a1, a2);
    V m = V{a0.x - T(0.5) * t.x, a0.y - T(0.5) * t.y};
    V d = csub(a1, a2);
    // s = d * (DIR i sqrt3/2)
    const T s3 = T(S3);
    V s = crot<DIR>(V{d.x * s3, d.y * s3});
    v[0] = cadd(a0, t);
    v[1] = cadd(m, s);
    v[2] = csub(m, s);
}

// 5 points: with t1 = a1 + a4, t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3,
// X1,4 = a0 + c1 t1 + c2 t2 +- DIR i (s1 t3 + s2 t4) and
// X2,3 = a0 + c2 t1 + c1 t2 +- DIR i (s2 t3 - s1 t4), c_k = cos(2 pi k / 5),
// s_k = sin(2 pi k / 5).
template <int DIR, typename V> __device__ __forceinline__ void dft5(V* v)
{
    using T = decltype(v[0].x);
    constexpr double C1 = 0.30901699437494742410;   // cos(2 pi / 5)
    constexpr double C2 = -0.80901699437494742410;  // cos(4 pi / 5)
    constexpr double S1 = 0.95105651629515357212;   // sin(2 pi / 5)
    constexpr double S2 = 0.58778525229247312917;   // sin(4 pi / 5)
    const T c1 = T(C1), c2 = T(C2), s1 = T(S1), s2 = T(S2);
    const V a0 = v[0];
    const V t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]), t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const V m1 = V{a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y};
    const V m2 = V{a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y};
    const V u1 = crot<DIR>(V{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
    const V u2 = crot<DIR>(V{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
    v[0] = V{a0.x + t1.x + t2.x, a0.y + t1.y + t2.y};
    v[1] = cadd(m1, u1);
    v[4] = csub(m1, u1);
    v[2] = cadd(m2, u2);
    v[3] = csub(m2, u2);
}

template <int DIR, typename V> __device__ __forceinline__ void dft8(V* v)
{
    V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    V o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4v<DIR>(e0, e1, e2, e3);
    dft4v<DIR>(o0, o1, o2, o3);
    o1 = w16<DIR, 2>(o1);
    o2 = w16<DIR, 4>(o2);
    o3 = w16<DIR, 6>(o3);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
template <int DIR, typename V> __device__ __forceinline__ void dft16(V* v)
{
    V y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        V a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
        dft4v<DIR>(a0, a1, a2, a3);
        y[n2][0] = a0;
        y[n2][1] = a1;
        y[n2][2] = a2;
        y[n2][3] = a3;
    }
    y[1][1] = w16<DIR, 1>(y[1][1]);
    y[1][2] = w16<DIR, 2>(y[1][2]);
    y[1][3] = w16<DIR, 3>(y[1][3]);
    y[2][1] = w16<DIR, 2>(y[2][1]);
    y[2][2] = w16<DIR, 4>(y[2][2]);
    y[2][3] = w16<DIR, 6>(y[2][3]);
    y[3][1] = w16<DIR, 3>(y[3][1]);
    y[3][2] = w16<DIR, 6>(y[3][2]);
    y[3][3] = w16<DIR, 9>(y[3][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        V a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
        dft4v<DIR>(a0, a1, a2, a3);
        v[k1] = a0;
        v[k1 + 4] = a1;
        v[k1 + 8] = a2;
        v[k1 + 12] = a3;
    }
}

// a * exp(DIR * 2 pi i * M / 32), M odd in [1, 16): constants cos/sin(M pi / 16)
template <int DIR, int M, typename V> __device__ __forceinline__ V w32(V a)
{
    using T = decltype(a.x);
    if constexpr (M % 2 == 0) return w16<DIR, M / 2>(a);
    else {
        // cos(k pi/16), k = 1, 3, 5, ..., 15
        constexpr double C[8] = {0.98078528040323044913, 0.83146961230254523708, 0.55557023301960222474,
                                 0.19509032201612826785, -0.19509032201612826785, -0.55557023301960222474,
                                 -0.83146961230254523708, -0.98078528040323044913};
        constexpr double S[8] = {0.19509032201612826785, 0.55557023301960222474, 0.83146961230254523708,
                                 0.98078528040323044913, 0.98078528040323044913, 0.83146961230254523708,
                                 0.55557023301960222474, 0.19509032201612826785};
        constexpr double cr = C[M / 2];
        constexpr double ci = DIR < 0 ? -S[M / 2] : S[M / 2];
        const T c = T(cr), s = T(ci);
        return V{a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

template <int DIR, int K = 1, typename V> __device__ __forceinline__ void static_for32(V* o)
{
    if constexpr (K < 16) {
        o[K] = w32<DIR, K>(o[K]);
        static_for32<DIR, K + 1>(o);
    }
}

// 32 = 2 x 16 (decimation in time): X[k] = E[k] + w^k O[k], X[k+16] = E[k] - w^k O[k].
template <int DIR, typename V> __device__ __forceinline__ void dft32(V* v)
{
    V e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        e[i] = v[2 * i];
        o[i] = v[2 * i + 1];
    }
    dft16<DIR>(e);
    dft16<DIR>(o);
    static_for32<DIR>(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 16] = csub(e[k], o[k]);
    }
}

template <int R, int DIR, typename V> __device__ __forceinline__ void dft(V* v);

// Compile-time cos and sin of the angle 2 pi m / n (double precision,
// rounded once to T where used): the angle is folded into [0, pi/2] by the
// symmetries of sin and cos and summed as Taylor series.  The twiddles of
// in-register DFTs whose length is not covered by the constants above.
constexpr double ct_pi = 3.14159265358979323846264338327950288;
constexpr double ct_sin_series(double x)
{
    double term = x, sum = x;
    for (int k = 1; k < 20; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos_series(double x)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 20; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// m in (-n/2, n/2]: angle 2 pi m / n in (-pi, pi]
constexpr int ct_fold(int m, int n)
{
    m %= n;
    if (m < 0) m += n;
    if (2 * m > n) m -= n;
    return m;
}
constexpr double ct_cos_2pi(int m, int n)
{
    const int a = ct_fold(m, n) < 0 ? -ct_fold(m, n) : ct_fold(m, n);  // cos is even
    // angle 2 pi a / n in [0, pi]; beyond pi/2 use cos(x) = -cos(pi - x)
    return 4 * a <= n ? ct_cos_series(2.0 * ct_pi * a / n) : -ct_cos_series(ct_pi * (n - 2 * a) / n);
}
constexpr double ct_sin_2pi(int m, int n)
{
    const int f = ct_fold(m, n), a = f < 0 ? -f : f;
    const double v = 4 * a <= n ? ct_sin_series(2.0 * ct_pi * a / n) : ct_sin_series(ct_pi * (n - 2 * a) / n);
    return f < 0 ? -v : v;  // sin is odd; sin(x) = sin(pi - x)
}
template <int I, int N, class F> __device__ __forceinline__ void ct_loop(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        ct_loop<I + 1, N>(f);
    }
}

// Cooley-Tukey DFT of length N1 N2 in registers, for factors that share a
// prime (9 = 3 x 3, 25 = 5 x 5, 27 = 3 x 9): n = N2 n1 + n2, k = k1 + N1 k2;
// N2 DFTs of length N1 along n1, the twiddles w^(n2 k1) (w = exp(DIR 2 pi i
// / N1 N2)), then N1 DFTs of length N2 along n2.
template <int DIR, int N1, int N2, typename V> __device__ __forceinline__ void dft_ct(V* v)
{
    using T = decltype(v[0].x);
    constexpr int N = N1 * N2;
    V a[N2][N1];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) a[n2][n1] = v[N2 * n1 + n2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) dft<N1, DIR>(a[n2]);
    ct_loop<1, N2>([&](auto i2) {
        constexpr int n2 = decltype(i2)::value;
        ct_loop<1, N1>([&](auto i1) {
            constexpr int k1 = decltype(i1)::value;
            constexpr double c = ct_cos_2pi(n2 * k1, N), sn = DIR * ct_sin_2pi(n2 * k1, N);
            V& x = a[n2][k1];
            x = V{x.x * T(c) - x.y * T(sn), x.x * T(sn) + x.y * T(c)};
        });
    });
    V b[N2];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) b[n2] = a[n2][k1];
        dft<N2, DIR>(b);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) v[k1 + N1 * k2] = b[k2];
    }
}

// Prime-factor (Good-Thomas) DFT of length N1 N2 with gcd(N1, N2) = 1: no
// twiddle factors.  Inputs are read at j = (N2 j1 + N1 j2) mod N into an
// N1 x N2 array, N2 DFTs of length N1 run along j1 and N1 DFTs of length N2
// along j2, and the result (k1, k2) is X[(E1 k1 + E2 k2) mod N] with
// E1 = N2 (N2^-1 mod N1) and E2 = N1 (N1^-1 mod N2), because then
// j k = N2 E1 j1 k1 + N1 E2 j2 k2 (mod N) and N2 E1 = 1 (mod N1),
// N1 E2 = 1 (mod N2).
constexpr int inv_mod(int a, int m)
{
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}
template <int DIR, int N1, int N2, typename V> __device__ __forceinline__ void dft_pfa(V* v)
{
    constexpr int N = N1 * N2;
    constexpr int E1 = N2 * inv_mod(N2 % N1, N1), E2 = N1 * inv_mod(N1 % N2, N2);
    V a[N2][N1];
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2)
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) a[j2][j1] = v[(N2 * j1 + N1 * j2) % N];
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) dft<N1, DIR>(a[j2]);
    V b[N1][N2];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) b[k1][j2] = a[j2][k1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) dft<N2, DIR>(b[k1]);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) v[(E1 * k1 + E2 * k2) % N] = b[k1][k2];
}

template <int R, int DIR, typename V> __device__ __forceinline__ void dft(V* v)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 3) dft3<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else if constexpr (R == 5) dft5<DIR>(v);
    else if constexpr (R == 6) dft_pfa<DIR, 2, 3>(v);
    else if constexpr (R == 10) dft_pfa<DIR, 2, 5>(v);
    else if constexpr (R == 12) dft_pfa<DIR, 4, 3>(v);
    else if constexpr (R == 15) dft_pfa<DIR, 3, 5>(v);
    else if constexpr (R == 20) dft_pfa<DIR, 4, 5>(v);
    else if constexpr (R == 24) dft_pfa<DIR, 8, 3>(v);
    else if constexpr (R == 30) dft_pfa<DIR, 2, 15>(v);
    else if constexpr (R == 9) dft_ct<DIR, 3, 3>(v);
    else if constexpr (R == 25) dft_ct<DIR, 5, 5>(v);
    else if constexpr (R == 27) dft_ct<DIR, 3, 9>(v);
    else if constexpr (R == 8) dft8<DIR>(v);
    else if constexpr (R == 16) dft16<DIR>(v);
    else if constexpr (R == 32) dft32<DIR>(v);
    else static_assert(R == 2, "unsupported radix");
}

}  // namespace ps
