#pragma once
// Solution of one system from its stored elimination (the factor-only mode of
// solve_system: the eliminated matrix column-major with its rows in pivot
// order, and the pivots' reciprocals r_k), for a right-hand side given in
// pivot order, by one wave.  It replays the elimination's own operations on
// the right-hand side: for step k, y_q = fma(-l_qk, y_k, y_q) with
// l_qk = a_qk r_k at the positions q > k (rows not yet pivoted at step k;
// a_qk is column k as step k found it, which the stored matrix holds there);
// then back substitution from the last unknown, z_k = y_k r_k and
// y_q = fma(-u_qk, z_k, y_q) for q < k.  The unknowns are therefore bit for
// bit those of eliminating the system with this right-hand side.
//
// Positions q = lane + 64 r sit on lanes (R slots); each stored element is
// read once (8 M^2 bytes per solve), with the columns fetched CK steps ahead
// into registers (double buffered) so that a block's loads are in flight
// while the previous block runs (a larger CK keeps more bytes in flight per
// wave, for launches with few waves, at the cost of 4 CK R registers).
#include "dev_util.h"

namespace rbfsl {

// y: the right-hand side at this lane's positions (pivot order); out(kk, zk)
// is called for every unknown kk from M-1 down to 0, zk wave-uniform.
template <int R, int CK = 8, typename Out>
__device__ __forceinline__ void replay_solve(const double *F, const double *rinv, const int M,
                                             const int lane, double (&y)[R], Out &&out) {
    double cb[CK][R], nb[CK][R];
    double cr[CK], nr[CK];  // the reciprocals of the same steps, fetched with the columns
    // forward: the elimination's updates of the right-hand side; positions
    // at or before k are pivoted rows (multiplier 0)
    auto fetch_fwd = [&](double (&buf)[CK][R], double (&rb)[CK], int k0) SI {
        sfor<0, CK>([&](auto CI) SI {
            constexpr int c = CI;
            const int kk = k0 + c;
            rb[c] = (kk < M) ? rinv[kk] : 0.0;
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                const int q = lane + 64 * r;
                double v = 0.0;
                if (q > kk && q < M) v = F[(int64_t)kk * M + q];
                buf[c][r] = v;
            });
        });
    };
    fetch_fwd(nb, nr, 0);
    for (int k0 = 0; k0 < M; k0 += CK) {
        sfor<0, CK>([&](auto CI) SI {
            cr[CI] = nr[CI];
            sfor<0, R>([&](auto RI) SI { cb[CI][RI] = nb[CI][RI]; });
        });
        if (k0 + CK < M) fetch_fwd(nb, nr, k0 + CK);
        sfor<0, CK>([&](auto CI) SI {
            constexpr int c = CI;
            const int kk = k0 + c;
            if (kk < M) {
                const double rk = cr[c];
                const int pl = kk & 63, pr = kk >> 6;
                double yp = bcast_d(y[0], pl);
                sfor<1, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    const double yr = bcast_d(y[r], pl);
                    yp = (pr == r) ? yr : yp;
                });
                sfor<0, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    const int q = lane + 64 * r;
                    const double l = (q <= kk) ? 0.0 : cb[c][r] * rk;
                    y[r] = fma(-l, yp, y[r]);
                });
            }
        });
    }
    // back substitution
    auto fetch_bwd = [&](double (&buf)[CK][R], double (&rb)[CK], int k1) SI {  // steps k1, k1-1, ...
        sfor<0, CK>([&](auto CI) SI {
            constexpr int c = CI;
            const int kk = k1 - c;
            rb[c] = (kk >= 0) ? rinv[kk] : 0.0;
            sfor<0, R>([&](auto RI) SI {
                constexpr int r = RI;
                const int q = lane + 64 * r;
                double v = 0.0;
                if (q < kk) v = F[(int64_t)kk * M + q];
                buf[c][r] = v;
            });
        });
    };
    fetch_bwd(nb, nr, M - 1);
    for (int k1 = M - 1; k1 >= 0; k1 -= CK) {
        sfor<0, CK>([&](auto CI) SI {
            cr[CI] = nr[CI];
            sfor<0, R>([&](auto RI) SI { cb[CI][RI] = nb[CI][RI]; });
        });
        if (k1 - CK >= 0) fetch_bwd(nb, nr, k1 - CK);
        sfor<0, CK>([&](auto CI) SI {
            constexpr int c = CI;
            const int kk = k1 - c;
            if (kk >= 0) {
                const double rk = cr[c];
                const int pl = kk & 63, pr = kk >> 6;
                double yk = bcast_d(y[0], pl);
                sfor<1, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    const double yr = bcast_d(y[r], pl);
                    yk = (pr == r) ? yr : yk;
                });
                const double zk = yk * rk;
                out(kk, zk);
                sfor<0, R>([&](auto RI) SI {
                    constexpr int r = RI;
                    const int q = lane + 64 * r;
                    const double yn = fma(-cb[c][r], zk, y[r]);
                    y[r] = (q < kk) ? yn : y[r];
                });
            }
        });
    }
}

}  // namespace rbfsl
