// Givens update of one Hessenberg column and the least-squares right-hand side
// (complex GMRES), and the back substitution on the triangle; device code shared
// by the single and the batched solvers.
#pragma once

#include <hip/hip_runtime.h>

namespace h2 {

// col (length j + 2) holds h_0..h_j and h_{j+1} = ||w||; apply rotations 0..j-1,
// form rotation j (cs[j], sn[j]) that zeroes h_{j+1}, update g; returns |g_{j+1}|.
__device__ inline double givens_column(double2* col, int j, double* cs, double2* sn, double2* g) {
    for (int i = 0; i < j; ++i) {   // previous rotations: [c s; -conj(s) c] [a; b]
        const double2 a = col[i], b = col[i + 1];
        const double c = cs[i];
        const double2 s = sn[i];
        col[i] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
        col[i + 1] = make_double2(-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y);
    }
    const double2 a = col[j], b = col[j + 1];
    const double aa = hypot(a.x, a.y), bb = hypot(b.x, b.y);
    double c;
    double2 s, r;
    if (bb == 0.0) {
        c = 1.0; s = make_double2(0, 0); r = a;
    } else if (aa == 0.0) {
        c = 0.0; s = make_double2(1.0, 0.0); r = b;
    } else {
        const double rho = hypot(aa, bb);
        c = aa / rho;
        const double2 ph = make_double2(a.x / aa, a.y / aa);          // a / |a|
        s = make_double2((ph.x * b.x + ph.y * b.y) / rho, (ph.y * b.x - ph.x * b.y) / rho);  // ph * conj(b) / rho
        r = make_double2(ph.x * rho, ph.y * rho);
    }
    cs[j] = c;
    sn[j] = s;
    col[j] = r;
    col[j + 1] = make_double2(0, 0);
    const double2 gj = g[j];
    // g_{j+1} = -conj(s) g_j ; g_j = c g_j
    g[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[j] = make_double2(c * gj.x, c * gj.y);
    return hypot(g[j + 1].x, g[j + 1].y);
}

// y = R^-1 g on the leading k x k triangle of H (column major, leading dimension ldh)
__device__ inline void back_substitute(const double2* H, int ldh, int k, const double2* g, double2* y) {
    for (int i = k - 1; i >= 0; --i) {
        double2 s = g[i];
        for (int q = i + 1; q < k; ++q) {
            const double2 h = H[(int64_t)q * ldh + i], yq = y[q];
            s.x -= h.x * yq.x - h.y * yq.y;
            s.y -= h.x * yq.y + h.y * yq.x;
        }
        const double2 d = H[(int64_t)i * ldh + i];
        const double den = d.x * d.x + d.y * d.y;
        y[i] = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
    }
}

}  // namespace h2
