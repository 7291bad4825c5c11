// Krylov drivers (Linear System / Solvers section: restarted GMRES(m),
// BiCGSTAB; FGMRES for the learned preconditioner) and the preconditioner /
// solve entry points.
//
// GMRES(m): right preconditioned (Saad & Schultz 1986), classical
// Gram-Schmidt applied twice (CGS2) on the device with fused multi-dot /
// update kernels, or the same two passes with the second delayed by a step
// (DCGS2: one reduction and two reads of the basis per step), Givens
// rotations on the host (at most 61 scalars per step).
// BiCGSTAB: right preconditioned (van der Vorst 1992), fused vector updates
// and dot products.  The reported residual is always recomputed in FP64 as
// ||b - A x|| / ||b||.  Vectors live in the tile-lane layout for the whole
// solve; b and x are permuted once on entry and exit.
#include "rsv_internal.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

struct SolverWork {
    double *pool = nullptr;   // nvec * nv doubles, zero-initialised (phantom slots stay zero)
    int nvec = 0;
};

static rsv_status ws_reserve(rsv_matrix *M, int nvec)
{
    rsv_ctx *c = M->g->ctx;
    if (!M->ws) {
        M->ws = new (std::nothrow) SolverWork();
        if (!M->ws) return set_err(c, RSV_ERR_OOM, "workspace");
    }
    SolverWork *w = M->ws;
    if (w->nvec >= nvec) return RSV_OK;
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    dev_free(w->pool);
    w->pool = nullptr;
    w->nvec = 0;
    const size_t bytes = (size_t)nvec * (size_t)M->nv * sizeof(double);
    rsv_status s = dev_alloc(c, (void **)&w->pool, bytes);
    if (s != RSV_OK) return s;
    RSV_HIP(c, hipMemsetAsync(w->pool, 0, bytes, c->stream));
    w->nvec = nvec;
    return RSV_OK;
}

static void ws_free(rsv_matrix *M)
{
    if (M->ws) {
        dev_free(M->ws->pool);
        delete M->ws;
        M->ws = nullptr;
    }
}

namespace {

struct Ctl {
    double tol, rtol, atol;
    double nb = 0.0, r0 = -1.0;
    bool met(double rn) const
    {
        if (rn <= tol * nb) return true;
        if (rtol > 0.0 && r0 >= 0.0 && rn <= rtol * r0) return true;
        if (atol > 0.0 && rn <= atol) return true;
        return false;
    }
};

// z = M^{-1} v for the solver (identity when M is NULL)
static rsv_status pc_apply(rsv_ctx *c, PcImpl *P, int64_t n, const double *v, double *z)
{
    if (!P) return launch_copy(c, n, v, z);
    return P->apply(v, z);
}

// Apply previous rotations to h[0..j+1] and form the new one (same
// convention as the oracle: a zero column keeps the residual estimate).
static void givens_step(int j, double *h, double *cs, double *sn, double *g)
{
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
    }
    const double a = h[j], b = h[j + 1];
    const double rr = std::hypot(a, b);
    double cc = 0.0, ss = 1.0;
    if (rr > 0.0) { cc = a / rr; ss = b / rr; }
    cs[j] = cc;
    sn[j] = ss;
    h[j] = rr;
    h[j + 1] = 0.0;
    g[j + 1] = -ss * g[j];
    g[j] = cc * g[j];
}

struct Solve {
    rsv_matrix *M;
    rsv_ctx *c;
    const Geo *geo;
    int64_t n;
    Ctl ctl;
    std::vector<double> *hist;
    bool record;
    rsv_stats *st;
};

// r = b - A x into r, returns ||r||
static rsv_status true_resid(Solve &S, const double *b, const double *x, double *r, double *rn)
{
    rsv_status s = mat_spmv(S.M, SPMV_RESID, x, r, b, 0, 0, SC_RR);
    if (s == RSV_OK) s = scal_to_host(S.c, SC_RR, 1);
    if (s != RSV_OK) return s;
    *rn = std::sqrt(S.c->h_scal[SC_RR]);
    return RSV_OK;
}

static rsv_status gmres(Solve &S, PcImpl *P, PcImpl *FB, double theta, int m, int64_t maxit, bool flexible,
                        bool dcgs, double *b, double *x, double *pool)
{
    rsv_ctx *c = S.c;
    const int64_t n = S.n;
    double *V = pool;                                         // (m+1) vectors
    double *Z = pool + (int64_t)(m + 1) * n;                   // FGMRES: m vectors
    double *zt = pool + (int64_t)(flexible ? 2 * m + 1 : m + 1) * n;
    double *ut = zt + n;
    const double nb = S.ctl.nb;
    rsv_status rc = RSV_OK;
    int64_t its = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m + 1, 0.0), sn(m + 1, 0.0), g(m + 2, 0.0), y(m, 0.0);
    auto Hc = [&](int col, int row) -> double & { return H[(size_t)col * (m + 1) + row]; };
    int consecutive_fb = 0;
    for (;;) {
        double beta;
        rsv_status s = true_resid(S, b, x, V, &beta);
        if (s != RSV_OK) return s;
        const double relres = beta / nb;
        if (!std::isfinite(relres)) return set_err(c, RSV_ERR_NAN, "non-finite residual");
        if (its == 0) {
            S.ctl.r0 = beta;
            if (S.record) S.hist->push_back(relres);
        }
        S.st->final_relres = relres;
        if (S.ctl.met(beta)) { rc = RSV_OK; break; }
        if (its >= maxit) { rc = RSV_NOT_CONVERGED; break; }
        s = launch_axpby(c, n, 1.0 / beta, V, 0.0, V);
        if (s != RSV_OK) return s;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        bool fb_rest = false;
        consecutive_fb = 0;
        if (!flexible && dcgs) {
            // DCGS2.  Step j leaves V[j] final and V[j + 1] once projected
            // and normalised (tentative); its Hessenberg column is tentative
            // until step j + 1 has measured how far V[j + 1] was from the
            // span of V[0..j] (dots s = V[0..j]^T V[j + 1]).  With
            // V[j + 1] = sum_i s_i V_i + beta q_{j+1}, the final column j is
            // h + gamma s on rows 0..j and gamma beta on row j + 1, and the
            // product of the tentative vector projects as
            // A M^-1 q_{j+1} = (w - Q Hbar s) / beta, so its column is
            // (u - Hbar s) / beta with u = Q^T w.  The convergence test of a
            // step uses its tentative column; a stopping step keeps it (its
            // basis vectors V[0..j] are all final).  Speculation as for CGS2:
            // a discarded step writes only V[j + 1], V[j + 2] and scratch.
            auto enqueue = [&](int j) -> rsv_status {
                double *w = V + (int64_t)(j + 1) * n;
                rsv_status e = pc_apply(c, P, n, V + (int64_t)j * n, zt);
                if (e == RSV_OK) e = mat_spmv(S.M, SPMV_NORM, zt, w, nullptr, 0, 0, SC_W0);
                if (e == RSV_OK) e = launch_dcgs_dots(c, n, V, n, j + 1, w, SC_DP);
                if (e == RSV_OK) e = launch_dcgs_update(c, n, V, n, j + 1, w, SC_DP);
                if (e == RSV_OK) e = scal_to_host_async(c, j & 1, SC_DP, 2 * (j + 1) + 4);
                return e;
            };
            std::vector<double> Hraw((size_t)(m + 1) * m, 0.0), ht(m + 2, 0.0), hc(m + 2, 0.0);
            std::vector<double> cs_t(m + 1), sn_t(m + 1), g_t(m + 2);
            auto Hr = [&](int col, int row) -> double & { return Hraw[(size_t)col * (m + 1) + row]; };
            double gam_prev = 0.0, est = beta;
            if ((s = enqueue(0)) != RSV_OK) return s;
            for (int j = 0; j < m; ++j) {
                const bool ahead = j + 1 < m && its + 1 < maxit && !S.ctl.met(0.25 * est);
                if (ahead && (s = enqueue(j + 1)) != RSV_OK) return s;
                if ((s = scal_wait(c, j & 1)) != RSV_OK) return s;
                const int K = j + 1;
                const double *d = c->h_spec + (size_t)(j & 1) * SC_COUNT + SC_DP;
                const double bj = d[2 * K], uj = d[2 * K + 1], d2 = d[2 * K + 2], om = d[2 * K + 3];
                bool finite = std::isfinite(bj) && std::isfinite(uj) && std::isfinite(d2) && std::isfinite(om);
                for (int i = 0; i < 2 * K; ++i) finite = finite && std::isfinite(d[i]);
                if (!finite) return set_err(c, RSV_ERR_NAN, "non-finite Arnoldi column");
                if (j >= 1) {
                    // column j - 1 becomes final; rotate it with the final rotations
                    for (int i = 0; i < j; ++i) Hr(j - 1, i) = ht[i] + gam_prev * d[i];
                    Hr(j - 1, j) = gam_prev * bj;
                    std::fill(hc.begin(), hc.end(), 0.0);
                    for (int i = 0; i <= j; ++i) hc[i] = Hr(j - 1, i);
                    givens_step(j - 1, hc.data(), cs.data(), sn.data(), g.data());
                    for (int i = 0; i <= j; ++i) Hc(j - 1, i) = hc[i];
                }
                const bool happy = !(d2 > DCGS_LOST * om);
                const double gam = happy ? 0.0 : std::sqrt(d2) / bj;
                std::fill(ht.begin(), ht.end(), 0.0);
                for (int k = 0; k <= j; ++k) {
                    double a = (k < j) ? d[K + k] : uj;
                    for (int i = 0; i < j; ++i) a -= Hr(i, k) * d[i];
                    ht[k] = a / bj;
                }
                ht[j + 1] = gam;
                hc = ht;
                cs_t = cs;
                sn_t = sn;
                g_t = g;
                givens_step(j, hc.data(), cs_t.data(), sn_t.data(), g_t.data());
                ++its;
                jdone = j + 1;
                est = std::fabs(g_t[j + 1]);
                if (S.record) S.hist->push_back(est / nb);
                if (!std::isfinite(est)) return set_err(c, RSV_ERR_NAN, "non-finite residual estimate");
                if (S.ctl.met(est) || its >= maxit || happy || j + 1 == m) {
                    for (int i = 0; i <= j + 1; ++i) Hc(j, i) = hc[i];
                    cs = cs_t;
                    sn = sn_t;
                    g = g_t;
                    break;
                }
                gam_prev = gam;
                if (!ahead && (s = enqueue(j + 1)) != RSV_OK) return s;
            }
        } else if (!flexible) {
            // The host's work on step j (Givens rotation, convergence test)
            // overlaps the device's step j + 1, which is enqueued before step
            // j's scalars are awaited -- except when the estimate is within a
            // factor 4 of the target, where that step would most likely be
            // discarded.  A discarded step only wrote V[j + 2], the
            // preconditioner's scratch and scalar slots no later step reads.
            auto enqueue = [&](int j) -> rsv_status {
                double *w = V + (int64_t)(j + 1) * n;
                rsv_status e = pc_apply(c, P, n, V + (int64_t)j * n, zt);
                if (e == RSV_OK) e = mat_spmv(S.M, SPMV_NORM, zt, w, nullptr, 0, 0, SC_W0);
                if (e == RSV_OK) e = launch_mdot(c, n, V, n, j + 1, w, SC_H1);
                if (e == RSV_OK) e = launch_upd_dot(c, n, V, n, j + 1, w, SC_H1, SC_H2);
                if (e == RSV_OK) e = launch_upd_norm(c, n, V, n, j + 1, w, SC_H1, SC_H2, SC_HN);
                if (e == RSV_OK) e = launch_scale_dev(c, n, w, SC_HN);
                if (e == RSV_OK) e = scal_to_host_async(c, j & 1, 0, SC_H2 + j + 1);
                return e;
            };
            double est = beta;
            if ((s = enqueue(0)) != RSV_OK) return s;
            std::vector<double> hcol(m + 2, 0.0);
            for (int j = 0; j < m; ++j) {
                const bool ahead = j + 1 < m && its + 1 < maxit && !S.ctl.met(0.25 * est);
                if (ahead && (s = enqueue(j + 1)) != RSV_OK) return s;
                if ((s = scal_wait(c, j & 1)) != RSV_OK) return s;
                const double *hs = c->h_spec + (size_t)(j & 1) * SC_COUNT;
                std::fill(hcol.begin(), hcol.end(), 0.0);
                for (int i = 0; i <= j; ++i) hcol[i] = hs[SC_H1 + i] + hs[SC_H2 + i];
                const double hn = std::sqrt(hs[SC_HN]);
                const double w0 = std::sqrt(hs[SC_W0]);
                hcol[j + 1] = hn;
                bool finite = std::isfinite(hn) && std::isfinite(w0);
                for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(hcol[i]);
                if (!finite) return set_err(c, RSV_ERR_NAN, "non-finite Arnoldi column");
                givens_step(j, hcol.data(), cs.data(), sn.data(), g.data());
                for (int i = 0; i <= j + 1; ++i) Hc(j, i) = hcol[i];
                const bool happy = (hn <= 1e-14 * w0);
                ++its;
                jdone = j + 1;
                est = std::fabs(g[j + 1]);
                if (S.record) S.hist->push_back(est / nb);
                if (!std::isfinite(est)) return set_err(c, RSV_ERR_NAN, "non-finite residual estimate");
                if (S.ctl.met(est) || its >= maxit || happy) break;
                if (!ahead && j + 1 < m && (s = enqueue(j + 1)) != RSV_OK) return s;
            }
        }
        for (int j = 0; flexible && j < m; ++j) {
            double *w = V + (int64_t)(j + 1) * n;
            double *z = flexible ? Z + (int64_t)j * n : zt;
            std::vector<double> cs_save(cs), sn_save(sn), g_save(g);
            std::vector<double> hcol(m + 2, 0.0);
            bool used_fb = false, happy = false, accepted = false;
            for (int attempt = 0; attempt < 2 && !accepted; ++attempt) {
                const bool want_fb = flexible && (fb_rest || attempt == 1);
                PcImpl *use = want_fb ? FB : P;
                used_fb = want_fb;
                s = pc_apply(c, use, n, V + (int64_t)j * n, z);
                if (s != RSV_OK) return s;
                s = mat_spmv(S.M, SPMV_NORM, z, w, nullptr, 0, 0, SC_W0);
                if (s == RSV_OK) s = launch_mdot(c, n, V, n, j + 1, w, SC_H1);
                if (s == RSV_OK) s = launch_upd_dot(c, n, V, n, j + 1, w, SC_H1, SC_H2);
                if (s == RSV_OK) s = launch_upd_norm(c, n, V, n, j + 1, w, SC_H1, SC_H2, SC_HN);
                if (s == RSV_OK) s = launch_scale_dev(c, n, w, SC_HN);
                if (s == RSV_OK) s = scal_to_host(c, 0, SC_H2 + j + 1);
                if (s != RSV_OK) return s;
                const double *hs = c->h_scal;
                for (int i = 0; i <= j; ++i) hcol[i] = hs[SC_H1 + i] + hs[SC_H2 + i];
                const double hn = std::sqrt(hs[SC_HN]);
                const double w0 = std::sqrt(hs[SC_W0]);
                hcol[j + 1] = hn;
                bool finite = std::isfinite(hn) && std::isfinite(w0);
                for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(hcol[i]);
                if (!finite) {
                    if (flexible && !want_fb) continue;   // discard, recompute with the fallback
                    return set_err(c, RSV_ERR_NAN, "non-finite Arnoldi column");
                }
                cs = cs_save;
                sn = sn_save;
                g = g_save;
                std::vector<double> hc(hcol);
                givens_step(j, hc.data(), cs.data(), sn.data(), g.data());
                if (flexible && !want_fb && std::fabs(g[j + 1]) > theta * std::fabs(g_save[j])) continue;
                for (int i = 0; i <= j + 1; ++i) Hc(j, i) = hc[i];
                happy = (hn <= 1e-14 * w0);
                accepted = true;
            }
            if (!accepted) return set_err(c, RSV_ERR_NAN, "no acceptable Arnoldi column");
            if (flexible) {
                if (used_fb) { S.st->fallbacks++; consecutive_fb++; } else consecutive_fb = 0;
                if (consecutive_fb >= 3) fb_rest = true;
            }
            ++its;
            jdone = j + 1;
            const double est = std::fabs(g[j + 1]);
            if (S.record) S.hist->push_back(est / nb);
            if (!std::isfinite(est)) return set_err(c, RSV_ERR_NAN, "non-finite residual estimate");
            if (S.ctl.met(est) || its >= maxit || happy) break;
        }
        for (int i = jdone - 1; i >= 0; --i) {
            double sacc = g[i];
            for (int q = i + 1; q < jdone; ++q) sacc -= Hc(q, i) * y[q];
            y[i] = (Hc(i, i) != 0.0) ? sacc / Hc(i, i) : 0.0;
        }
        s = scal_set(c, SC_Y, y.data(), jdone);
        if (s != RSV_OK) return s;
        if (flexible) {
            s = launch_combine(c, n, Z, n, jdone, SC_Y, x, 1);
        } else {
            s = launch_combine(c, n, V, n, jdone, SC_Y, ut, 0);
            if (s == RSV_OK) s = pc_apply(c, P, n, ut, zt);
            if (s == RSV_OK) s = launch_axpby(c, n, 1.0, zt, 1.0, x);
        }
        if (s != RSV_OK) return s;
        S.st->restarts++;
    }
    S.st->its = its;
    return rc;
}

static rsv_status bicgstab(Solve &S, PcImpl *P, int64_t maxit, double *b, double *x, double *pool)
{
    rsv_ctx *c = S.c;
    const int64_t n = S.n;
    double *r = pool, *rh = pool + n, *p = pool + 2 * n, *v = pool + 3 * n, *ph = pool + 4 * n;
    double *s_ = pool + 5 * n, *sh = pool + 6 * n, *t = pool + 7 * n;
    const double nb = S.ctl.nb;
    double rn;
    rsv_status s = true_resid(S, b, x, r, &rn);
    if (s != RSV_OK) return s;
    S.ctl.r0 = rn;
    if (S.record) S.hist->push_back(rn / nb);
    S.st->final_relres = rn / nb;
    if (!std::isfinite(rn)) return set_err(c, RSV_ERR_NAN, "non-finite residual");
    int64_t its = 0;
    rsv_status rc = RSV_OK;
    if (!S.ctl.met(rn)) {
        if ((s = launch_copy(c, n, r, rh)) != RSV_OK) return s;
        if ((s = launch_axpby(c, n, 0.0, r, 0.0, p)) != RSV_OK) return s;
        if ((s = launch_axpby(c, n, 0.0, r, 0.0, v)) != RSV_OK) return s;
        const double nrh = rn;
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        double rho_new = rn * rn;   // rhat = r0
        double nr = rn;
        {
            double vals[2] = {rn * rn, rho_new};
            if ((s = scal_set(c, SC_RR, vals, 2)) != RSV_OK) return s;
        }
        for (;;) {
            if (its >= maxit) { rc = RSV_NOT_CONVERGED; break; }
            if (!(std::fabs(rho_new) >= 1e-300 * nrh * nr)) { rc = RSV_BREAKDOWN; break; }
            const double beta = (rho_new / rho) * (alpha / omega);
            if ((s = launch_bicg_p(c, n, r, v, beta, omega, p)) != RSV_OK) return s;
            if ((s = pc_apply(c, P, n, p, ph)) != RSV_OK) return s;
            if ((s = mat_spmv(S.M, SPMV_DOT1, ph, v, rh, 0, 0, SC_RV)) != RSV_OK) return s;
            if ((s = launch_bicg_s(c, n, r, v, s_, SC_RH, SC_RV, SC_SS)) != RSV_OK) return s;
            if ((s = scal_to_host_async(c, 0, SC_RR, SC_SS - SC_RR + 1)) != RSV_OK) return s;
            // The second half's preconditioner apply and product depend only
            // on s, so they are enqueued before the mid-iteration scalars are
            // awaited (and discarded when ||s|| already meets the tolerance),
            // except within a factor 4 of the target.
            const bool ahead = !S.ctl.met(0.25 * nr);
            if (ahead) {
                if ((s = pc_apply(c, P, n, s_, sh)) != RSV_OK) return s;
                if ((s = mat_spmv(S.M, SPMV_DOT2, sh, t, s_, 0, 0, SC_TS)) != RSV_OK) return s;
            }
            if ((s = scal_wait(c, 0)) != RSV_OK) return s;
            const double rv = c->h_spec[SC_RV];
            if (!std::isfinite(rv)) return set_err(c, RSV_ERR_NAN, "non-finite rhat.v");
            if (rv == 0.0) { rc = RSV_BREAKDOWN; break; }
            alpha = rho_new / rv;
            const double sn_ = std::sqrt(c->h_spec[SC_SS]);
            if (S.ctl.met(sn_)) {
                if ((s = launch_axpby(c, n, alpha, ph, 1.0, x)) != RSV_OK) return s;
                ++its;
                double tr;
                if ((s = true_resid(S, b, x, r, &tr)) != RSV_OK) return s;
                if (S.record) S.hist->push_back(tr / nb);
                S.st->final_relres = tr / nb;
                if (S.ctl.met(tr)) { rc = RSV_OK; break; }
                rho = rho_new;
                if ((s = launch_dot(c, n, rh, r, SC_RH)) != RSV_OK) return s;
                if ((s = scal_to_host(c, SC_RH, 1)) != RSV_OK) return s;
                rho_new = c->h_scal[SC_RH];
                nr = tr;
                continue;
            }
            if (!ahead) {
                if ((s = pc_apply(c, P, n, s_, sh)) != RSV_OK) return s;
                if ((s = mat_spmv(S.M, SPMV_DOT2, sh, t, s_, 0, 0, SC_TS)) != RSV_OK) return s;
            }
            if ((s = launch_bicg_xr(c, n, alpha, 0.0, ph, sh, s_, t, rh, x, r, SC_RR)) != RSV_OK) return s;
            if ((s = scal_to_host(c, SC_RR, SC_TT - SC_RR + 1)) != RSV_OK) return s;
            const double tt = c->h_scal[SC_TT];
            omega = (tt > 0.0) ? c->h_scal[SC_TS] / tt : 0.0;
            rho = rho_new;
            rho_new = c->h_scal[SC_RH];
            nr = std::sqrt(c->h_scal[SC_RR]);
            ++its;
            if (S.record) S.hist->push_back(nr / nb);
            if (!std::isfinite(nr)) return set_err(c, RSV_ERR_NAN, "non-finite residual");
            if (S.ctl.met(nr)) {
                double tr;
                if ((s = true_resid(S, b, x, r, &tr)) != RSV_OK) return s;
                S.st->final_relres = tr / nb;
                if (S.ctl.met(tr)) { rc = RSV_OK; break; }
                if ((s = launch_dot(c, n, rh, r, SC_RH)) != RSV_OK) return s;
                if ((s = scal_to_host(c, SC_RH, 1)) != RSV_OK) return s;
                rho_new = c->h_scal[SC_RH];
                nr = tr;
            }
            if (omega == 0.0) { rc = RSV_BREAKDOWN; break; }
        }
    }
    S.st->its = its;
    double tr;
    s = true_resid(S, b, x, t, &tr);
    if (s != RSV_OK) return s;
    S.st->final_relres = tr / nb;
    return rc;
}

}  // namespace

extern "C" {

rsv_status rsv_precond_setup(rsv_matrix *A, const rsv_pc_params *p, rsv_precond **out, int64_t *bad_cell)
{
    if (!A || !p || !out) return set_err(A ? A->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (bad_cell) *bad_cell = -1;
    rsv_ctx *c = A->g->ctx;
    if (p->precision != RSV_FP64 && p->precision != RSV_FP32) return set_err(c, RSV_ERR_ARG, "bad precision");
    if (p->iluk_level < 0 || p->iluk_level > 8) return set_err(c, RSV_ERR_ARG, "iluk_level must be in [0, 8]");
    if (p->iluk_level > 0 && (A->bs == 1 || (p->type != RSV_PC_BILU0 && p->type != RSV_PC_RAS &&
                                             p->type != RSV_PC_CPR)))
        return set_err(c, RSV_ERR_ARG, "ILU(k) with k > 0 is a block BILU / RAS local solver");
    if (A->bs == 1 && p->type == RSV_PC_LEARNED)
        return set_err(c, RSV_ERR_ARG, "the learned preconditioner needs a 3x3-block matrix");
    if (p->local_solver != RSV_LOCAL_ILUK && p->local_solver != RSV_LOCAL_ILUT)
        return set_err(c, RSV_ERR_ARG, "bad local_solver");
    if (p->local_solver == RSV_LOCAL_ILUT &&
        (A->bs == 1 || p->iluk_level != 0 ||
         (p->type != RSV_PC_BILU0 && p->type != RSV_PC_RAS && p->type != RSV_PC_CPR)))
        return set_err(c, RSV_ERR_ARG, "ILUT is a block BILU / RAS local solver (iluk_level 0)");
    if (p->type == RSV_PC_CPR) {
        if (A->bs == 1) return set_err(c, RSV_ERR_ARG, "CPR needs a 3x3-block matrix");
        if (p->cpr_stage != RSV_PC_BILU0 && p->cpr_stage != RSV_PC_RAS)
            return set_err(c, RSV_ERR_ARG, "cpr_stage must be RSV_PC_BILU0 or RSV_PC_RAS");
        if (p->cpr_variant < RSV_CPR_FP || p->cpr_variant > RSV_CPR_FFPF)
            return set_err(c, RSV_ERR_ARG, "bad cpr_variant");
        if (p->cpr_decouple < RSV_DECOUPLE_NONE || p->cpr_decouple > RSV_DECOUPLE_ABF)
            return set_err(c, RSV_ERR_ARG, "bad cpr_decouple");
        if (p->mg_pre < 1 || p->mg_pre > 8 || p->mg_post < 1 || p->mg_post > 8)
            return set_err(c, RSV_ERR_ARG, "mg_pre and mg_post must be in [1, 8]");
        if (p->mg_coarse < 1 || p->mg_coarse > 1024) return set_err(c, RSV_ERR_ARG, "mg_coarse must be in [1, 1024]");
    }
    rsv_precond *P = new (std::nothrow) rsv_precond();
    if (!P) return set_err(c, RSV_ERR_OOM, "precond");
    P->A = A;
    P->p = *p;
    rsv_status s = RSV_OK;
    switch (p->type) {
    case RSV_PC_NONE: break;
    case RSV_PC_BILU0:
        s = (A->bs == 1) ? sras_create(A, p, &P->impl, bad_cell)
            : (p->local_solver == RSV_LOCAL_ILUT) ? rasT_create(A, p, &P->impl, bad_cell)
            : (p->iluk_level > 0) ? rasK_create(A, p, &P->impl, bad_cell) : bilu0_create(A, p, &P->impl, bad_cell);
        break;
    case RSV_PC_RAS:
        s = (A->bs == 1) ? sras_create(A, p, &P->impl, bad_cell)
            : (p->local_solver == RSV_LOCAL_ILUT) ? rasT_create(A, p, &P->impl, bad_cell)
            : (p->iluk_level > 0) ? rasK_create(A, p, &P->impl, bad_cell) : ras_create(A, p, &P->impl, bad_cell);
        break;
    case RSV_PC_CPR: {
        rsv_pc_params st = *p;
        st.type = p->cpr_stage;
        PcImpl *stage = nullptr;
        s = (st.local_solver == RSV_LOCAL_ILUT) ? rasT_create(A, &st, &stage, bad_cell)
            : (st.iluk_level > 0) ? rasK_create(A, &st, &stage, bad_cell)
            : (st.type == RSV_PC_RAS) ? ras_create(A, &st, &stage, bad_cell) : bilu0_create(A, &st, &stage, bad_cell);
        if (s == RSV_OK) s = cpr_create(A, p, stage, &P->impl, bad_cell);
        break;
    }
    case RSV_PC_LEARNED: {
        rsv_pc_params fb = *p;
        fb.type = RSV_PC_BILU0;
        s = bilu0_create(A, &fb, &P->fallback, bad_cell);
        if (s == RSV_OK) s = learned_create(A, p, &P->impl, P->fallback);
        break;
    }
    default: s = set_err(c, RSV_ERR_ARG, "bad preconditioner type");
    }
    if (s != RSV_OK) {
        rsv_precond_destroy(P);
        return s;
    }
    *out = P;
    return RSV_OK;
}

void rsv_precond_destroy(rsv_precond *P)
{
    if (!P) return;
    if (P->A) (void)hipStreamSynchronize(P->A->g->ctx->stream);
    delete P->impl;
    delete P->fallback;
    delete P;
}

int64_t rsv_precond_apply_bytes(const rsv_precond *P)
{
    if (!P || !P->impl) return -1;
    return P->impl->apply_bytes();
}

rsv_status rsv_precond_bilu0_factors(const rsv_precond *P, double *L, double *Dinv)
{
    if (!P || !L || !Dinv) return set_err(P ? P->A->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    if (P->p.type != RSV_PC_BILU0) return set_err(P->A->g->ctx, RSV_ERR_ARG, "not a BILU0 preconditioner");
    return P->impl->bilu0_factors(L, Dinv);
}

rsv_status rsv_spmv(rsv_matrix *M, double alpha, const double *x, double beta, double *y)
{
    if (!M || !x || !y) return set_err(M ? M->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_ctx *c = M->g->ctx;
    if (M->bs == 1) {
        // a scalar matrix works on row-ordered vectors: one launch, no staging
        rsv_status s = mat_spmv(M, SPMV_AXPBY, x, y, nullptr, alpha, beta, 0);
        if (s == RSV_OK) {
            hipError_t e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
        }
        return s;
    }
    // the tile-lane copies of x and A x live in the solver workspace (no allocation per call)
    rsv_status s = ws_reserve(M, 2);
    if (s != RSV_OK) return s;
    const int64_t n = M->g->nv;
    double *xt = M->ws->pool, *yt = M->ws->pool + n;
    s = launch_nat_to_tl(c, M->g->geo, x, xt);
    if (s == RSV_OK) s = launch_spmv(c, M->g->geo, M->d_A, SPMV_Y, xt, yt, nullptr, 1.0, 0.0, 0);
    if (s == RSV_OK) s = launch_tl_to_nat(c, M->g->geo, yt, y, alpha, beta);
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
    }
    return s;
}

rsv_status rsv_axpby(rsv_ctx *c, int64_t n, double alpha, const double *x, double beta, double *y)
{
    if (!c || !x || !y || n < 0) return set_err(c, RSV_ERR_ARG, "bad argument");
    if (n == 0) return RSV_OK;
    return launch_axpby(c, n, alpha, x, beta, y);
}

rsv_status rsv_spmv_noalloc(rsv_matrix *M, double alpha, const double *x, double beta, double *y)
{
    if (!M || !x || !y) return set_err(M ? M->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_ctx *c = M->g->ctx;
    if (M->bs == 1) return rsv_spmv(M, alpha, x, beta, y);   // scalar: no scratch at all
    const int64_t n = M->g->nv;
    if (!c->d_scratch) return set_err(c, RSV_ERR_ARG, "no fixed scratch on this device");
    if (2 * n > NOALLOC_SCRATCH_DOUBLES)
        return set_err(c, RSV_ERR_ARG, "grid too large for the fixed scratch (" + std::to_string(16 * n) + " > " +
                                           std::to_string((long long)RSV_NOALLOC_SCRATCH_BYTES) + " bytes)");
    // the same kernels as rsv_spmv, on the fixed scratch: x is laid out into
    // the first half (every slot written, absent cells as zero), A x into the
    // second (every slot written), then read back into y
    double *xt = c->d_scratch, *yt = c->d_scratch + n;
    rsv_status s = launch_nat_to_tl(c, M->g->geo, x, xt);
    if (s == RSV_OK) s = launch_spmv(c, M->g->geo, M->d_A, SPMV_Y, xt, yt, nullptr, 1.0, 0.0, 0);
    if (s == RSV_OK) s = launch_tl_to_nat(c, M->g->geo, yt, y, alpha, beta);
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
    }
    return s;
}

rsv_status rsv_precond_apply(rsv_precond *P, const double *r, double *z)
{
    if (!P || !r || !z) return set_err(P ? P->A->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_matrix *M = P->A;
    rsv_ctx *c = M->g->ctx;
    rsv_status s = ws_reserve(M, 2);
    if (s == RSV_OK) s = flags_reset(c);
    if (s != RSV_OK) return s;
    const int64_t n = M->nv;
    double *rt = M->ws->pool, *zt = M->ws->pool + n;
    s = mat_in(M, r, rt);
    if (s == RSV_OK) s = pc_apply(c, P->impl, n, rt, zt);
    if (s == RSV_OK) s = mat_out(M, zt, z, 1.0, 0.0);
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
        s = flags_check(c, nullptr);
    }
    return s;
}

rsv_status rsv_solve(rsv_matrix *A, rsv_precond *P, const rsv_solver_params *p, const double *b, double *x,
                     rsv_stats *st)
{
    rsv_stats dummy;
    if (!st) st = &dummy;
    std::memset(st, 0, sizeof(*st));
    st->bad_cell = -1;
    if (!A || !p || !b || !x) return st->status = set_err(A ? A->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_ctx *c = A->g->ctx;
    auto t0 = std::chrono::steady_clock::now();
    if (P && P->A != A) return st->status = set_err(c, RSV_ERR_ARG, "preconditioner built on another matrix");
    const int m = p->restart;
    if ((p->method == RSV_GMRES || p->method == RSV_FGMRES) && (m < 1 || m > 60))
        return st->status = set_err(c, RSV_ERR_ARG, "restart must be in [1, 60]");
    if (p->method != RSV_GMRES && p->method != RSV_FGMRES && p->method != RSV_BICGSTAB)
        return st->status = set_err(c, RSV_ERR_ARG, "bad method");
    if (p->ortho != RSV_CGS2 && p->ortho != RSV_DCGS2) return st->status = set_err(c, RSV_ERR_ARG, "bad ortho");
    if (p->maxit < 0 || !(p->tol >= 0.0)) return st->status = set_err(c, RSV_ERR_ARG, "bad tol/maxit");
    PcImpl *impl = P ? P->impl : nullptr;
    if (P && P->p.type == RSV_PC_LEARNED && p->method != RSV_FGMRES)
        return st->status = set_err(c, RSV_ERR_ARG, "the learned preconditioner needs FGMRES");
    // FGMRES with a fixed preconditioner uses that preconditioner as its own fallback
    const int nvec = (p->method == RSV_BICGSTAB) ? 10 : (p->method == RSV_FGMRES ? 2 * m + 5 : m + 5);
    rsv_status s = ws_reserve(A, nvec);
    if (s != RSV_OK) return st->status = s;
    const int64_t n = A->nv;
    double *pool = A->ws->pool;
    double *bt = pool + (int64_t)(nvec - 2) * n;
    double *xt = pool + (int64_t)(nvec - 1) * n;
    s = mat_in(A, b, bt);
    if (s == RSV_OK) s = mat_in(A, x, xt);
    if (s == RSV_OK) s = launch_nonfinite(c, n, bt, SC_MISC);
    if (s == RSV_OK) s = launch_dot(c, n, bt, bt, SC_BB);
    if (s == RSV_OK) s = scal_to_host(c, 0, SC_MISC + 1);   // slots SC_BB and SC_MISC
    if (s != RSV_OK) return st->status = s;
    double bad = c->h_scal[SC_MISC];
    s = launch_nonfinite(c, n, xt, SC_MISC);
    if (s == RSV_OK) s = scal_to_host(c, SC_MISC, 1);
    if (s != RSV_OK) return st->status = s;
    if (bad != 0.0 || c->h_scal[SC_MISC] != 0.0)
        return st->status = set_err(c, RSV_ERR_NAN, "non-finite entries in b or x0");
    s = flags_reset(c);
    if (s != RSV_OK) return st->status = s;
    Solve S{A, c, &A->g->geo, n, Ctl{p->tol, p->rtol, p->atol}, &A->hist, p->record_history != 0, st};
    A->hist.clear();
    S.ctl.nb = std::sqrt(c->h_scal[SC_BB]);
    rsv_status rc;
    if (S.ctl.nb == 0.0) {
        // b = 0: x = 0 is the answer
        s = launch_axpby(c, n, 0.0, bt, 0.0, xt);
        if (s != RSV_OK) return st->status = s;
        if (S.record) A->hist.push_back(0.0);
        rc = RSV_OK;
    } else if (p->method == RSV_BICGSTAB) {
        rc = bicgstab(S, impl, p->maxit, bt, xt, pool);
    } else {
        const bool flex = (p->method == RSV_FGMRES);
        PcImpl *fb = (P && P->fallback) ? P->fallback : impl;
        rc = gmres(S, impl, fb, P ? P->p.theta : 0.99, m, p->maxit, flex, !flex && p->ortho == RSV_DCGS2, bt, xt,
                   pool);
    }
    if (rc < 0) return st->status = rc;
    s = mat_out(A, xt, x, 1.0, 0.0);
    if (s == RSV_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
    }
    if (s == RSV_OK) s = flags_check(c, &st->bad_cell);
    if (s != RSV_OK) return st->status = s;
    st->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st->status = rc;
    return rc;
}

int64_t rsv_solve_history(const rsv_matrix *A, double *hist, int64_t cap)
{
    if (!A) return 0;
    const int64_t n = (int64_t)A->hist.size();
    if (hist)
        for (int64_t i = 0; i < n && i < cap; ++i) hist[i] = A->hist[i];
    return n;
}

void rsv_matrix_destroy(rsv_matrix *M)
{
    if (!M) return;
    (void)hipStreamSynchronize(M->g->ctx->stream);
    ws_free(M);
    dev_free(M->d_A);
    dev_free(M->d_coef);
    delete M;
}

int64_t rsv_matrix_device_bytes(const rsv_matrix *M)
{
    if (!M) return 0;
    int64_t b = M->bytes;
    if (M->ws) b += (int64_t)M->ws->nvec * M->nv * (int64_t)sizeof(double);
    return b;
}

}  // extern "C"
