// Predicted gain variance of a selection (Sec. 2 gain uncertainty, eq. cov
// with eq. noisecov; eq. gaincov / eq. gaincov_v1 of Sec. 5.4): per
// antenna, E|g_est / g_true - 1|^2 = (SNR^-2 / 2) (diag C_eta + diag C_phi)
// for the logarithmic (logcal) form of the redundant-calibration system.
// Host only, FP64, computed once per selection.
//
// The logarithm splits eq. redcal into two real systems of the same
// sparsity, amplitude (ln|V_b| = eta_i + eta_j + A_alpha) and phase
// (arg V_b = phi_i - phi_j + psi_alpha).  Each equation carries noise
// variance SNR^-2 / 2, so a half's covariance is that times the inverse of
// its normal matrix H = A^T A.  H is singular along the degeneracies of
// Sec. 5.2 (one for amplitude, three for phase), and gains are compared
// after those are removed: C is the gains' block of any generalised inverse
// projected off span{1} (amplitude) or span{1, x, y} (phase) -- every
// solution differs by a null vector whose gain part lies in that span.
//
// Here the generalised inverse is the inverse of H with the degeneracies
// grounded: amplitude, the first type unknown removed; phase, antenna 0 and
// two types of independent displacement removed (their null-vector minor is
// nonsingular).  The remaining matrix is [[B, E], [E^T, F]] with B the N' x N'
// antenna block -- banded in raster order, half-width the largest raster
// offset of the selection (a signless graph Laplacian for amplitude, a
// grounded Laplacian for phase) -- E its coupling to the K' type unknowns
// and F = diag(N_alpha).  With S = F - E^T B^-1 E and W = B^-1 E:
//     C = B^-1 + W S^-1 W^T,
//     diag C = diag B^-1 + rowwise w^T S^-1 w,   C Q = B^-1 Q + W S^-1 W^T Q,
// diag B^-1 by the selected inversion of B = L D L^T inside the band, and
// diag(P C P)_i = C_ii - 2 (C Q)_i . Q_i + Q_i^T (Q^T C Q) Q_i for the
// orthonormal basis Q of the projected span.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "../../include/rrcal.h"

namespace {

// Symmetric positive-definite band matrix, lower half stored row-wise:
// a(i, j) for i - w <= j <= i.
struct Band {
    int m, w;
    std::vector<double> v;
    Band(int m_, int w_) : m(m_), w(w_), v((size_t)m_ * (w_ + 1), 0.0) {}
    double& at(int i, int j) { return v[(size_t)i * (w + 1) + (j - i + w)]; }
    double get(int i, int j) const {
        if (j > i) std::swap(i, j);
        if (i - j > w) return 0.0;
        return v[(size_t)i * (w + 1) + (j - i + w)];
    }
};

// In place: B = L D L^T (unit lower L in the band, D returned).  False if a
// pivot is not positive.
bool ldlt(Band& b, std::vector<double>& d) {
    const int m = b.m, w = b.w;
    d.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
        const int j0 = std::max(0, i - w);
        for (int j = j0; j < i; ++j) {
            double s = b.at(i, j);
            for (int k = std::max(j0, j - w); k < j; ++k) s -= b.at(i, k) * b.at(j, k) * d[k];
            b.at(i, j) = s / d[j];
        }
        double s = b.at(i, i);
        for (int k = j0; k < i; ++k) s -= b.at(i, k) * b.at(i, k) * d[k];
        if (!(s > 0.0)) return false;
        d[i] = s;
        b.at(i, i) = 1.0;
    }
    return true;
}

// x = B^-1 x with B = L D L^T from ldlt
void band_solve(const Band& f, const std::vector<double>& d, double* x) {
    const int m = f.m, w = f.w;
    for (int i = 0; i < m; ++i) {
        double s = x[i];
        for (int k = std::max(0, i - w); k < i; ++k) s -= f.v[(size_t)i * (w + 1) + (k - i + w)] * x[k];
        x[i] = s;
    }
    for (int i = 0; i < m; ++i) x[i] /= d[i];
    for (int i = m - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k <= std::min(m - 1, i + w); ++k) s -= f.v[(size_t)k * (w + 1) + (i - k + w)] * x[k];
        x[i] = s;
    }
}

// diag(B^-1) from the factors: Z = B^-1 satisfies Z = D^-1 L^-1 + (I - L^T) Z,
// so with rows taken from the last, Z(i, j) = -sum_{k > i} L(k, i) Z(k, j)
// (j > i) and Z(i, i) = 1 / D_i - sum_{k > i} L(k, i) Z(k, i); every Z entry
// needed lies inside the band.
std::vector<double> band_inverse_diag(const Band& f, const std::vector<double>& d) {
    const int m = f.m, w = f.w;
    Band z(m, w);
    auto L = [&](int k, int i) { return f.v[(size_t)k * (w + 1) + (i - k + w)]; };   // k > i
    auto Z = [&](int i, int j) -> double { return z.get(i, j); };
    for (int i = m - 1; i >= 0; --i) {
        const int kmax = std::min(m - 1, i + w);
        for (int j = kmax; j > i; --j) {
            double s = 0.0;
            for (int k = i + 1; k <= kmax; ++k) s -= L(k, i) * Z(k, j);
            z.at(j, i) = s;
        }
        double s = 1.0 / d[i];
        for (int k = i + 1; k <= kmax; ++k) s -= L(k, i) * Z(k, i);
        z.at(i, i) = s;
    }
    std::vector<double> out(m);
    for (int i = 0; i < m; ++i) out[i] = z.get(i, i);
    return out;
}

// Dense symmetric positive-definite solve (Cholesky), in place on rhs
// columns; false if not positive definite.
bool chol_solve(std::vector<double> a, int n, std::vector<double>& rhs, int ncol) {
    for (int j = 0; j < n; ++j) {
        double s = a[j * n + j];
        for (int k = 0; k < j; ++k) s -= a[j * n + k] * a[j * n + k];
        if (!(s > 0.0)) return false;
        a[j * n + j] = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = a[i * n + j];
            for (int k = 0; k < j; ++k) t -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = t / a[j * n + j];
        }
    }
    for (int c = 0; c < ncol; ++c) {
        double* x = &rhs[(size_t)c * n];
        for (int i = 0; i < n; ++i) {
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= a[i * n + k] * x[k];
            x[i] = s / a[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int k = i + 1; k < n; ++k) s -= a[k * n + i] * x[k];
            x[i] = s / a[i * n + i];
        }
    }
    return true;
}

// diag of the projected gains' covariance of one half (sign +1 amplitude,
// -1 phase), per unit noise variance of each equation.
bool half_diag(int n, const int32_t* xy, int K, int sign, std::vector<double>& out) {
    const int N = n * n;
    int bw = 0;
    for (int t = 0; t < K; ++t) bw = std::max(bw, xy[2 * t + 1] * n + std::abs(xy[2 * t]));
    // grounded unknowns
    int ant_drop = -1, t_drop0 = -1, t_drop1 = -1;
    if (sign > 0) {
        t_drop0 = 0;
    } else {
        ant_drop = 0;
        for (int a = 0; a < K && t_drop1 < 0; ++a)
            for (int b = a + 1; b < K; ++b)
                if (xy[2 * a] * xy[2 * b + 1] - xy[2 * a + 1] * xy[2 * b] != 0) {
                    t_drop0 = a;
                    t_drop1 = b;
                    break;
                }
        if (t_drop1 < 0) return false;
    }
    // antenna a -> row of B (the dropped antenna has none)
    auto brow = [&](int a) { return ant_drop >= 0 ? (a > ant_drop ? a - 1 : (a == ant_drop ? -1 : a)) : a; };
    const int m = ant_drop >= 0 ? N - 1 : N;
    std::vector<int> tcol(K, -1);
    int kp = 0;
    for (int t = 0; t < K; ++t)
        if (t != t_drop0 && t != t_drop1) tcol[t] = kp++;
    Band b(m, bw);
    std::vector<double> e((size_t)kp * m, 0.0), f(kp, 0.0);    // E column-major [kp][m]
    for (int t = 0; t < K; ++t) {
        const int dx = xy[2 * t], dy = xy[2 * t + 1];
        for (int y = dy; y < n; ++y)
            for (int x = std::max(0, dx); x < n + std::min(0, dx); ++x) {
                const int i = y * n + x, j = i - (dy * n + dx);
                const int ri = brow(i), rj = brow(j);
                if (ri >= 0) b.at(ri, ri) += 1.0;
                if (rj >= 0) b.at(rj, rj) += 1.0;
                if (ri >= 0 && rj >= 0) b.at(std::max(ri, rj), std::min(ri, rj)) += (double)sign;
                const int c = tcol[t];
                if (c >= 0) {
                    f[c] += 1.0;
                    if (ri >= 0) e[(size_t)c * m + ri] += 1.0;
                    if (rj >= 0) e[(size_t)c * m + rj] += (double)sign;
                }
            }
    }
    std::vector<double> d;
    if (!ldlt(b, d)) return false;
    // W = B^-1 E, S = F - E^T W
    std::vector<double> wm = e;
    for (int c = 0; c < kp; ++c) band_solve(b, d, &wm[(size_t)c * m]);
    std::vector<double> s((size_t)kp * kp, 0.0);
    for (int r = 0; r < kp; ++r)
        for (int c = 0; c < kp; ++c) {
            double acc = (r == c) ? f[r] : 0.0;
            for (int i = 0; i < m; ++i) acc -= e[(size_t)r * m + i] * wm[(size_t)c * m + i];
            s[r * kp + c] = acc;
        }
    // orthonormal basis Q of the projected span over all N antennas
    const int nq = sign > 0 ? 1 : 3;
    std::vector<double> q((size_t)nq * N);
    for (int a = 0; a < N; ++a) {
        q[a] = 1.0;
        if (nq == 3) {
            q[N + a] = a % n;
            q[2 * N + a] = a / n;
        }
    }
    for (int c = 0; c < nq; ++c) {                 // modified Gram-Schmidt
        for (int p = 0; p < c; ++p) {
            double dot = 0.0;
            for (int a = 0; a < N; ++a) dot += q[c * N + a] * q[p * N + a];
            for (int a = 0; a < N; ++a) q[c * N + a] -= dot * q[p * N + a];
        }
        double nn = 0.0;
        for (int a = 0; a < N; ++a) nn += q[c * N + a] * q[c * N + a];
        nn = std::sqrt(nn);
        for (int a = 0; a < N; ++a) q[c * N + a] /= nn;
    }
    // C Q = B^-1 Q + W S^-1 W^T Q (rows of the dropped antenna are zero)
    std::vector<double> bq((size_t)nq * m), wtq((size_t)nq * kp, 0.0);
    for (int c = 0; c < nq; ++c) {
        for (int a = 0; a < N; ++a)
            if (brow(a) >= 0) bq[(size_t)c * m + brow(a)] = q[c * N + a];
        for (int r = 0; r < kp; ++r) {
            double acc = 0.0;
            for (int i = 0; i < m; ++i) acc += wm[(size_t)r * m + i] * bq[(size_t)c * m + i];
            wtq[(size_t)c * kp + r] = acc;
        }
        band_solve(b, d, &bq[(size_t)c * m]);
    }
    std::vector<double> sw = wtq;                  // S^-1 W^T Q
    if (kp > 0 && !chol_solve(s, kp, sw, nq)) return false;
    std::vector<double> cq((size_t)nq * N, 0.0);
    for (int c = 0; c < nq; ++c)
        for (int a = 0; a < N; ++a) {
            const int i = brow(a);
            if (i < 0) continue;
            double acc = bq[(size_t)c * m + i];
            for (int r = 0; r < kp; ++r) acc += wm[(size_t)r * m + i] * sw[(size_t)c * kp + r];
            cq[c * N + a] = acc;
        }
    // Q^T C Q
    std::vector<double> qcq((size_t)nq * nq, 0.0);
    for (int r = 0; r < nq; ++r)
        for (int c = 0; c < nq; ++c) {
            double acc = 0.0;
            for (int a = 0; a < N; ++a) acc += q[r * N + a] * cq[c * N + a];
            qcq[r * nq + c] = acc;
        }
    // diag C = diag B^-1 + rowwise w^T S^-1 w
    std::vector<double> dz = band_inverse_diag(b, d);
    std::vector<double> sinv((size_t)kp * kp, 0.0);
    for (int r = 0; r < kp; ++r) sinv[(size_t)r * kp + r] = 1.0;
    if (kp > 0 && !chol_solve(s, kp, sinv, kp)) return false;
    out.assign(N, 0.0);
    for (int a = 0; a < N; ++a) {
        const int i = brow(a);
        double cii = 0.0;
        if (i >= 0) {
            cii = dz[i];
            for (int r = 0; r < kp; ++r) {
                double acc = 0.0;
                for (int c = 0; c < kp; ++c) acc += sinv[(size_t)r * kp + c] * wm[(size_t)c * m + i];
                cii += wm[(size_t)r * m + i] * acc;
            }
        }
        double v = cii;
        for (int c = 0; c < nq; ++c) v -= 2.0 * cq[c * N + a] * q[c * N + a];
        for (int r = 0; r < nq; ++r)
            for (int c = 0; c < nq; ++c) v += q[r * N + a] * qcq[r * nq + c] * q[c * N + a];
        out[a] = v;
    }
    return true;
}

}  // namespace

extern "C" {

int rrc_gain_variance(int32_t n, const int32_t* types_xy, int32_t k, double snr, double* var_out) {
    if (n < 2 || n > RRC_MAX_GRID || k < 1 || k > RRC_MAX_TYPES || !types_xy || !var_out || !(snr > 0.0))
        return RRC_EINVAL;
    int32_t na = 0, np = 0;
    const int rc = rrc_degeneracy_count(n, types_xy, k, &na, &np);
    if (rc != RRC_OK) return rc;
    if (na + np != 4) return RRC_EDEGEN;
    std::vector<double> ca, cp;
    if (!half_diag(n, types_xy, k, +1, ca) || !half_diag(n, types_xy, k, -1, cp)) return RRC_EDEGEN;
    const double s = 0.5 / (snr * snr);
    for (int a = 0; a < n * n; ++a) var_out[a] = s * (ca[a] + cp[a]);
    return RRC_OK;
}

}  // extern "C"
