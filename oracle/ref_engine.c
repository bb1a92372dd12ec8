/* Plain FP64 reference engine for the compiled-CUT-graph flow (oracle).
 *
 * TEST INFRASTRUCTURE ONLY: called by the oracle's Python wrapper for graphs too
 * large for the NumPy oracle.  Shares nothing with the GPU library.  Plain loops
 * in stored record order; OpenMP only over independent targets or sets.
 *
 * Layouts: records in target-grouped (CSR) form off[N+1], i[E], j[E], c[E];
 * operands eta[N][nsets], x/y[N][nops][nsets] (row-major).
 *
 *   apply      y_k = sum_{e in E(k)} c_e eta_{i_e} x_{j_e}      (Eq. graph-actions)
 *   adj_x      g_x[j] += sum_{e: j_e=j} c_e eta_{i_e} w_{k_e}   (graph-level adjoint)
 *   adj_eta    g_eta[i] += sum_{e: i_e=i} c_e sum_op w_{k_e} x_{j_e}
 *   g2         eta_S = N_S / Q_S with N_S = -sum_t c_t eps_{a_t} h_{p_t},
 *              Q_S = 4 sum_t eps_{a_t}^2 + delta^2 (stencil rows t of S)
 *   wegner     eta_k = sgn * sum_{e in E_eta(k)} c_e h_{i_e} h_{j_e}
 *   g1         eta_S = h_S / (2 sum_t |eps_{a_t}| + delta) over the stencil
 *              rows t of S (the pairs S flips); 0 on strings without any
 *   flow       classic RK4, fixed ds, set b frozen after n_b steps
 *   flow_adj   exact adjoint of the discrete RK4 map, checkpoint recompute
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <string.h>

/* ---------------------------------------------------------------- records --
 * Majorana records of the given targets, by brute force over the left input:
 * for target mask K and every registry string A, B = A xor K is kept when B has
 * degree 2 or 4 (in the registry) and |A & B| is odd (the two anticommute).
 * Factor of [i Gamma_A, Gamma_B] = c Gamma_K: c = 2 i^e with
 * e = 1 + t(|A|) + t(|B|) - t(|K|) + 2 inv(A, B), t(d) = d(d-1)/2 and
 * inv(A, B) = #{(a, b) in A x B : a > b} counted pair by pair.
 * Records of one target come out in ascending left input (= ascending (i, j)).
 * counts[t] = number of records of targets[t]; with ri == NULL only counts are
 * produced, otherwise records of target t are written from offsets[t]. */
static int popc(uint64_t x) { return __builtin_popcountll(x); }

static int64_t find_mask(const uint64_t* sorted, const int64_t* order, int64_t N, uint64_t q) {
    int64_t lo = 0, hi = N - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (sorted[mid] == q) return order[mid];
        if (sorted[mid] < q) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static double maj_coeff(uint64_t A, uint64_t B, int m) {
    int inv = 0;
    for (int a = 0; a < m; ++a)
        if ((A >> a) & 1)
            for (int b = 0; b < a; ++b)
                if ((B >> b) & 1) ++inv;
    int dA = popc(A), dB = popc(B), dK = popc(A ^ B);
    int e = 1 + dA * (dA - 1) / 2 + dB * (dB - 1) / 2 - dK * (dK - 1) / 2 + 2 * inv;
    e = ((e % 4) + 4) % 4;
    return e == 0 ? 2.0 : -2.0; /* e is even for anticommuting Hermitian strings */
}

int orc_maj_records(int m, int64_t N, const uint64_t* masks, const uint64_t* sorted, const int64_t* order,
                    const int64_t* targets, int64_t nt, int64_t* counts, const int64_t* offsets, int32_t* ri,
                    int32_t* rj, double* rc) {
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
    for (int64_t t = 0; t < nt; ++t) {
        const uint64_t K = masks[targets[t]];
        int64_t n = 0;
        for (int64_t a = 0; a < N; ++a) {
            const uint64_t A = masks[a], B = A ^ K;
            const int dB = popc(B);
            if ((dB != 2 && dB != 4) || (popc(A & B) & 1) == 0) continue;
            if (ri) {
                const int64_t j = find_mask(sorted, order, N, B);
                if (j < 0) bad = 1;
                ri[offsets[t] + n] = (int32_t)a;
                rj[offsets[t] + n] = (int32_t)j;
                rc[offsets[t] + n] = maj_coeff(A, B, m);
            }
            ++n;
        }
        counts[t] = n;
    }
    return bad;
}

typedef struct {
    int64_t N, nops, nsets;
    const int64_t* off; const int32_t* ri; const int32_t* rj; const double* rc;
    /* generator: kind 0 = G2 stencil, 1 = Wegner graph over E_eta, 2 = G1 (stencil pairs) */
    int kind;
    const int64_t* st_off; const int32_t* st_a; const int32_t* st_p; const double* st_c;
    const int32_t* pairs; double delta;
    const int64_t* eoff; const int32_t* ei; const int32_t* ej; const double* ec;
    double gsign;
} orc_graph;

void orc_apply(const orc_graph* g, const double* eta, const double* x, double* y) {
    const int64_t nops = g->nops, ns = g->nsets;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < g->N; ++k) {
        for (int64_t op = 0; op < nops; ++op)
            for (int64_t s = 0; s < ns; ++s) {
                double acc = 0.0;
                for (int64_t e = g->off[k]; e < g->off[k + 1]; ++e)
                    acc += g->rc[e] * eta[(int64_t)g->ri[e] * ns + s] *
                           x[((int64_t)g->rj[e] * nops + op) * ns + s];
                y[(k * nops + op) * ns + s] = acc;
            }
    }
}

/* out[j] += adjoint_x(eta, w); parallel over sets (each set scatters alone). */
void orc_adj_x(const orc_graph* g, const double* eta, const double* w, double* out) {
    const int64_t nops = g->nops, ns = g->nsets;
#pragma omp parallel for
    for (int64_t s = 0; s < ns; ++s)
        for (int64_t k = 0; k < g->N; ++k)
            for (int64_t e = g->off[k]; e < g->off[k + 1]; ++e)
                for (int64_t op = 0; op < nops; ++op)
                    out[((int64_t)g->rj[e] * nops + op) * ns + s] +=
                        g->rc[e] * eta[(int64_t)g->ri[e] * ns + s] * w[(k * nops + op) * ns + s];
}

/* out[i] += adjoint_eta(w, x) */
void orc_adj_eta(const orc_graph* g, const double* w, const double* x, double* out) {
    const int64_t nops = g->nops, ns = g->nsets;
#pragma omp parallel for
    for (int64_t s = 0; s < ns; ++s)
        for (int64_t k = 0; k < g->N; ++k)
            for (int64_t e = g->off[k]; e < g->off[k + 1]; ++e) {
                double t = 0.0;
                for (int64_t op = 0; op < nops; ++op)
                    t += w[(k * nops + op) * ns + s] * x[((int64_t)g->rj[e] * nops + op) * ns + s];
                out[(int64_t)g->ri[e] * ns + s] += g->rc[e] * t;
            }
}

/* eta from the Hamiltonian column h = z[:, 0, :] (strided by nops*nsets). */
static void gen_eta(const orc_graph* g, const double* z, double* eta) {
    const int64_t nops = g->nops, ns = g->nsets;
#define H(r, s) z[((int64_t)(r) * nops) * ns + (s)]
    if (g->kind == 0) {
#pragma omp parallel for
        for (int64_t S = 0; S < g->N; ++S)
            for (int64_t s = 0; s < ns; ++s) {
                double num = 0.0, q = 0.0;
                for (int64_t t = g->st_off[S]; t < g->st_off[S + 1]; ++t) {
                    double eps = H(g->pairs[g->st_a[t]], s);
                    num += -g->st_c[t] * eps * H(g->st_p[t], s);
                    q += 4.0 * eps * eps;
                }
                eta[S * ns + s] = (g->st_off[S + 1] > g->st_off[S]) ? num / (q + g->delta * g->delta)
                                                                   : 0.0;
            }
    } else if (g->kind == 2) {
#pragma omp parallel for
        for (int64_t S = 0; S < g->N; ++S)
            for (int64_t s = 0; s < ns; ++s) {
                double d = g->delta;
                for (int64_t t = g->st_off[S]; t < g->st_off[S + 1]; ++t) d += 2.0 * fabs(H(g->pairs[g->st_a[t]], s));
                eta[S * ns + s] = (g->st_off[S + 1] > g->st_off[S]) ? H(S, s) / d : 0.0;
            }
    } else {
#pragma omp parallel for
        for (int64_t k = 0; k < g->N; ++k)
            for (int64_t s = 0; s < ns; ++s) {
                double acc = 0.0;
                for (int64_t e = g->eoff[k]; e < g->eoff[k + 1]; ++e)
                    acc += g->ec[e] * H(g->ei[e], s) * H(g->ej[e], s);
                eta[k * ns + s] = g->gsign * acc;
            }
    }
#undef H
}

/* gh[N][nsets] += eta'(h)^T gbar */
static void gen_vjp(const orc_graph* g, const double* z, const double* gbar, double* gh) {
    const int64_t nops = g->nops, ns = g->nsets;
#define H(r, s) z[((int64_t)(r) * nops) * ns + (s)]
#pragma omp parallel for
    for (int64_t s = 0; s < ns; ++s) {
        if (g->kind == 0) {
            for (int64_t S = 0; S < g->N; ++S) {
                if (g->st_off[S + 1] == g->st_off[S]) continue;
                double num = 0.0, q = 0.0;
                for (int64_t t = g->st_off[S]; t < g->st_off[S + 1]; ++t) {
                    double eps = H(g->pairs[g->st_a[t]], s);
                    num += -g->st_c[t] * eps * H(g->st_p[t], s);
                    q += 4.0 * eps * eps;
                }
                q += g->delta * g->delta;
                double gb = gbar[S * ns + s];
                for (int64_t t = g->st_off[S]; t < g->st_off[S + 1]; ++t) {
                    int64_t pa = g->pairs[g->st_a[t]];
                    double eps = H(pa, s);
                    gh[(int64_t)g->st_p[t] * ns + s] += gb * (-g->st_c[t] * eps / q);
                    gh[pa * ns + s] += gb * (-g->st_c[t] * H(g->st_p[t], s) / q -
                                             num * 8.0 * eps / (q * q));
                }
            }
        } else if (g->kind == 2) {
            for (int64_t S = 0; S < g->N; ++S) {
                if (g->st_off[S + 1] == g->st_off[S]) continue;
                double d = g->delta;
                for (int64_t t = g->st_off[S]; t < g->st_off[S + 1]; ++t) d += 2.0 * fabs(H(g->pairs[g->st_a[t]], s));
                const double gb = gbar[S * ns + s];
                gh[S * ns + s] += gb / d;
                for (int64_t t = g->st_off[S]; t < g->st_off[S + 1]; ++t) {
                    const int64_t pa = g->pairs[g->st_a[t]];
                    const double e = H(pa, s);
                    gh[pa * ns + s] += -2.0 * (e > 0.0 ? 1.0 : e < 0.0 ? -1.0 : 0.0) * gb * H(S, s) / (d * d);
                }
            }
        } else {
            for (int64_t k = 0; k < g->N; ++k)
                for (int64_t e = g->eoff[k]; e < g->eoff[k + 1]; ++e) {
                    double w = g->gsign * g->ec[e] * gbar[k * ns + s];
                    gh[(int64_t)g->ei[e] * ns + s] += w * H(g->ej[e], s);
                    gh[(int64_t)g->ej[e] * ns + s] += w * H(g->ei[e], s);
                }
        }
    }
#undef H
}

static void rhs(const orc_graph* g, const double* z, double* eta, double* k) {
    gen_eta(g, z, eta);
    orc_apply(g, eta, z, k);
}

/* One RK4 step from z into zout for the sets with act[s] != 0. */
static void rk4(const orc_graph* g, const double* z, double* zout, double ds, const int* act,
                double* eta, double* kk, double* zs, double* acc) {
    const int64_t ns = g->nsets, M = g->N * g->nops * ns;
    static const double a[4] = {0.0, 0.5, 0.5, 1.0};
    static const double w[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    memcpy(acc, z, sizeof(double) * M);
    memcpy(zs, z, sizeof(double) * M);
    for (int st = 0; st < 4; ++st) {
        rhs(g, zs, eta, kk);
        for (int64_t q = 0; q < M; ++q) acc[q] += ds * w[st] * kk[q];
        if (st < 3)
            for (int64_t q = 0; q < M; ++q) zs[q] = z[q] + ds * a[st + 1] * kk[q];
    }
    for (int64_t q = 0; q < M; ++q) zout[q] = act[q % ns] ? acc[q] : z[q];
}

static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* Flows z in place; ckpt (nullable) receives z at steps 0, c, 2c, ... */
void orc_flow(const orc_graph* g, double* z, double ds, const int32_t* nsteps, int ckpt_every,
              double* ckpt) {
    const int64_t ns = g->nsets, M = g->N * g->nops * ns;
    int T = 0;
    for (int64_t s = 0; s < ns; ++s) T = nsteps[s] > T ? nsteps[s] : T;
    double *eta = dalloc(g->N * ns), *kk = dalloc(M), *zs = dalloc(M), *acc = dalloc(M),
           *zn = dalloc(M);
    int* act = (int*)calloc((size_t)ns, sizeof(int));
    int nck = 0;
    for (int t = 0; t < T; ++t) {
        if (ckpt && ckpt_every > 0 && t % ckpt_every == 0) memcpy(ckpt + (int64_t)(nck++) * M, z, sizeof(double) * M);
        for (int64_t s = 0; s < ns; ++s) act[s] = nsteps[s] > t;
        rk4(g, z, zn, ds, act, eta, kk, zs, acc);
        memcpy(z, zn, sizeof(double) * M);
    }
    free(eta); free(kk); free(zs); free(acc); free(zn); free(act);
}

/* out = J(Z)^T mu */
static void jt(const orc_graph* g, const double* Z, const double* mu, double* out, double* eta,
               double* geta, double* gh) {
    const int64_t nops = g->nops, ns = g->nsets, M = g->N * nops * ns;
    gen_eta(g, Z, eta);
    memset(out, 0, sizeof(double) * M);
    orc_adj_x(g, eta, mu, out);
    memset(geta, 0, sizeof(double) * g->N * ns);
    orc_adj_eta(g, mu, Z, geta);
    memset(gh, 0, sizeof(double) * g->N * ns);
    gen_vjp(g, Z, geta, gh);
    for (int64_t r = 0; r < g->N; ++r)
        for (int64_t s = 0; s < ns; ++s) out[(r * nops) * ns + s] += gh[r * ns + s];
}

/* lam: in dL/dz(end), out dL/dz(0). */
void orc_flow_adjoint(const orc_graph* g, const double* z0, double ds, const int32_t* nsteps,
                      int ckpt_every, double* lam) {
    const int64_t ns = g->nsets, M = g->N * g->nops * ns;
    int T = 0;
    for (int64_t s = 0; s < ns; ++s) T = nsteps[s] > T ? nsteps[s] : T;
    if (T == 0) return;
    int nblk = (T + ckpt_every - 1) / ckpt_every;
    double* ck = dalloc((int64_t)nblk * M);
    double* zz = dalloc(M);
    memcpy(zz, z0, sizeof(double) * M);
    orc_flow(g, zz, ds, nsteps, ckpt_every, ck);
    double *states = dalloc((int64_t)ckpt_every * M), *eta = dalloc(g->N * ns), *kk = dalloc(M),
           *zs = dalloc(M), *acc = dalloc(M), *Z2 = dalloc(M), *Z3 = dalloc(M), *Z4 = dalloc(M),
           *u = dalloc(4 * M), *mu = dalloc(M), *geta = dalloc(g->N * ns), *gh = dalloc(g->N * ns);
    int* act = (int*)calloc((size_t)ns, sizeof(int));
    for (int b = nblk - 1; b >= 0; --b) {
        int t0 = b * ckpt_every, t1 = t0 + ckpt_every < T ? t0 + ckpt_every : T;
        memcpy(states, ck + (int64_t)b * M, sizeof(double) * M);
        for (int t = t0; t < t1 - 1; ++t) {
            for (int64_t s = 0; s < ns; ++s) act[s] = nsteps[s] > t;
            rk4(g, states + (int64_t)(t - t0) * M, states + (int64_t)(t - t0 + 1) * M, ds, act, eta,
                kk, zs, acc);
        }
        for (int t = t1 - 1; t >= t0; --t) {
            const double* z = states + (int64_t)(t - t0) * M;
            rhs(g, z, eta, kk);
            for (int64_t q = 0; q < M; ++q) Z2[q] = z[q] + 0.5 * ds * kk[q];
            rhs(g, Z2, eta, kk);
            for (int64_t q = 0; q < M; ++q) Z3[q] = z[q] + 0.5 * ds * kk[q];
            rhs(g, Z3, eta, kk);
            for (int64_t q = 0; q < M; ++q) Z4[q] = z[q] + ds * kk[q];
            double *u1 = u, *u2 = u + M, *u3 = u + 2 * M, *u4 = u + 3 * M;
            for (int64_t q = 0; q < M; ++q) mu[q] = ds / 6.0 * lam[q];
            jt(g, Z4, mu, u4, eta, geta, gh);
            for (int64_t q = 0; q < M; ++q) mu[q] = ds / 3.0 * lam[q] + ds * u4[q];
            jt(g, Z3, mu, u3, eta, geta, gh);
            for (int64_t q = 0; q < M; ++q) mu[q] = ds / 3.0 * lam[q] + 0.5 * ds * u3[q];
            jt(g, Z2, mu, u2, eta, geta, gh);
            for (int64_t q = 0; q < M; ++q) mu[q] = ds / 6.0 * lam[q] + 0.5 * ds * u2[q];
            jt(g, z, mu, u1, eta, geta, gh);
            for (int64_t q = 0; q < M; ++q)
                if (nsteps[q % ns] > t) lam[q] += u1[q] + u2[q] + u3[q] + u4[q];
        }
    }
    free(ck); free(zz); free(states); free(eta); free(kk); free(zs); free(acc); free(Z2); free(Z3);
    free(Z4); free(u); free(mu); free(geta); free(gh); free(act);
}
