// Host construction of the dyadic piecewise-polynomial approximations of Phi^{-1}.
//
// Section 2.1 (Figure 1; Lemma 2.2 piecewise linear, Lemma 2.3 piecewise cubic) uses
// polynomial pieces on intervals that shrink geometrically towards the tails.  Here:
// 16 intervals of (0, 1/2] -- I_j = [2^-(j+1), 2^-j) for j = 1..15 and I_16 = (0, 2^-16) --
// with one polynomial of degree d in the local coordinate t in [0, 1) per interval,
// chosen to minimise int_0^1 (Phi^{-1}(u(t)) - q_j(t))^2 dt, i.e. the mean squared error
// of Z~ against Z under the uniform law restricted to I_j.  The fit solves the normal
// equations H c = m (Hilbert matrix, moments of Phi^{-1} against 1, t, ..., t^d) in long
// double; the moments use Gauss-Legendre quadrature (composite and geometrically graded
// towards t = 0 on I_16, where Phi^{-1} has its logarithmic singularity), and Phi^{-1} is
// obtained by Halley iteration on Phi(z) = u with erfcl.
#include <cmath>
#include <cstring>

namespace mlmc {

namespace {

constexpr int kGauss = 48;

struct GaussRule {
    long double x[kGauss];  // nodes on [0, 1]
    long double w[kGauss];  // weights on [0, 1]
    GaussRule() {
        // roots of the Legendre polynomial P_n by Newton's method from Chebyshev guesses
        const int n = kGauss;
        for (int i = 0; i < n; ++i) {
            long double z = std::cos(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
            long double dp = 0;
            for (int it = 0; it < 100; ++it) {
                long double p0 = 1, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1);
                const long double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-21L) break;
            }
            {
                long double p0 = 1, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1);
            }
            x[i] = (1 - z) / 2;
            w[i] = 1 / ((1 - z * z) * dp * dp);  // = (2 / ((1 - z^2) P'^2)) / 2
        }
    }
};

// Phi^{-1}(u) for 0 < u < 1/2 in long double.
long double phi_inv_ld(long double u) {
    // starting value: the rational approximation of Abramowitz and Stegun, 26.2.23
    const long double s = std::sqrt(-2 * std::log(u));
    long double z = -(s - (2.515517L + 0.802853L * s + 0.010328L * s * s) /
                              (1 + 1.432788L * s + 0.189269L * s * s + 0.001308L * s * s * s));
    const long double rsqrt2 = 0.707106781186547524400844362104849039L;
    const long double rsqrt2pi = 0.398942280401432677939946059934381868L;
    for (int it = 0; it < 20; ++it) {
        const long double f = 0.5L * std::erfc(-z * rsqrt2) - u;
        const long double d = rsqrt2pi * std::exp(-0.5L * z * z);
        const long double e = f / d;
        const long double step = e / (1 + 0.5L * z * e);  // Halley
        z -= step;
        if (std::fabs(step) <= 1e-20L * std::fabs(z)) break;
    }
    return z;
}

// int_a^b f(u(t)) t^i dt for i = 0..d with the Gauss rule mapped to [a, b]
template <typename UofT>
void moments_on(const GaussRule& g, long double a, long double b, UofT u_of_t, int d, long double* m) {
    const long double h = b - a;
    for (int k = 0; k < kGauss; ++k) {
        const long double t = a + h * g.x[k];
        const long double f = phi_inv_ld(u_of_t(t)) * g.w[k] * h;
        long double tp = 1;
        for (int i = 0; i <= d; ++i) {
            m[i] += f * tp;
            tp *= t;
        }
    }
}

bool solve(int n, long double A[4][4], long double* b, long double* x) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0) return false;
        for (int k = 0; k < n; ++k) std::swap(A[c][k], A[piv][k]);
        std::swap(b[c], b[piv]);
        for (int r = c + 1; r < n; ++r) {
            const long double f = A[r][c] / A[c][c];
            for (int k = c; k < n; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        long double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
    return true;
}

}  // namespace

// out[16][4]: rows c_0..c_d of each interval (unused columns zero).  Returns false on a
// numerical failure (never expected).
bool build_l2_table(int degree, double out[16][4]) {
    static const GaussRule g;
    std::memset(out, 0, sizeof(double) * 16 * 4);
    for (int j = 1; j <= 16; ++j) {
        long double m[4] = {0, 0, 0, 0};
        if (j < 16) {
            const long double lo = std::ldexp(1.0L, -(j + 1));
            moments_on(g, 0, 1, [lo](long double t) { return lo * (1 + t); }, degree, m);
        } else {
            const long double sc = std::ldexp(1.0L, -16);
            // geometric grading towards the singular end: [2^-(k+1), 2^-k], k = 0..99
            for (int k = 0; k < 100; ++k)
                moments_on(g, std::ldexp(1.0L, -(k + 1)), std::ldexp(1.0L, -k),
                           [sc](long double t) { return sc * t; }, degree, m);
        }
        long double H[4][4];
        for (int a = 0; a <= degree; ++a)
            for (int b = 0; b <= degree; ++b) H[a][b] = 1.0L / (a + b + 1);
        long double c[4] = {0, 0, 0, 0};
        if (!solve(degree + 1, H, m, c)) return false;
        for (int i = 0; i <= degree; ++i) out[j - 1][i] = (double)c[i];
    }
    return true;
}

// Cell means of Phi^{-1} on 2^bits equal cells of (0, 1), lower half (n = 2^(bits-1) cells):
// with u = Phi(z), int_a^b Phi^{-1}(u) du = phi(Phi^{-1}(a)) - phi(Phi^{-1}(b)), so the mean
// of cell [a, b) is 2^bits (phi(z_a) - phi(z_b)).  The difference is formed without
// cancellation as phi(z_b) expm1((z_b - z_a)(z_b + z_a) / 2); phi(z_0) = 0 at a = 0 and
// z = 0 at b = 1/2.  Returns false on a numerical failure (never expected).
bool build_pconst_table(int bits, double* out) {
    if (bits < 1 || bits > 20) return false;
    const int n = 1 << (bits - 1);
    const long double scale = std::ldexp(1.0L, bits);
    const long double rsqrt2pi = 0.398942280401432677939946059934381868L;
    long double za = 0;  // Phi^{-1} of the cell's lower end (unused for the first cell)
    for (int i = 0; i < n; ++i) {
        const long double zb = (i + 1 == n) ? 0.0L : phi_inv_ld((i + 1) / scale);
        const long double pb = rsqrt2pi * std::exp(-0.5L * zb * zb);
        const long double diff = i == 0 ? -pb : pb * std::expm1(0.5L * (zb - za) * (zb + za));
        out[i] = (double)(scale * diff);
        if (!std::isfinite(out[i])) return false;
        za = zb;
    }
    return true;
}

}  // namespace mlmc
