// Coarse-spatial-mesh lanes of the engine (propagator PT_COARSE_MESH).
// Included by pt_engine.hip inside its anonymous namespace: it uses the
// engine's group barrier, flags, reductions and group vectors.
//
// The coarse propagators of Sec. 7.3 / Sec. 8 as this library reads them: the
// coarse mesh has nx/2 x ny/2 elements, coarse node (I, J) is fine node
// (2I, 2J), R is injection and P the bilinear interpolant (0 at fine Dirichlet
// nodes). A coarse step solves (C_c/dtau + K_c) x = C_c/dtau u + load with u
// the coarse input, the load being q(tau_{n+1}) f_c (primal) or P^T of the fine
// source of Eq. 4.6 at T_m, m = M(n-1)+1 (adjoint); its output is P x, and the
// primal theta follows Alg. 1 with dtau, N_tau from P x.
//
// Two lane kinds run these steps inside a pass's single engine launch:
//  * CM_GK_*: one batched step G(R u^k_n) of slice n (first warm iteration),
//    queued with the fine lanes; it writes the coarse output row Gk[n] (and
//    Gk_th[n]) and sets the slice's FL_GK flag;
//  * CM_SWEEP_*: the sequential correction sweep of Eq. 4.10 / Eq. 4.14 on the
//    coarse mesh, hat u_{n+1} = G(hat u_n) + R F_n - G(R u^k_n), hat u_1 = R F_0
//    (adjoint: downwards from R F_{N_tau}), on a group of its own. Each step
//    starts as soon as the batched step it reads is done and takes F_n only
//    when it needs it (after its solve), so the sweep overlaps the fine lanes.
//    Its outputs G(hat u_n) go to Gn[n], the primal theta chain to out_th and
//    Gn_th. In a cold launch (LaunchInfo::cold, the lane alone) the same lane
//    runs the cold sweep u^0_{n+1} = G(u^0_n) from u^0_0 = 0 (adjoint:
//    v^0_{n-1} = G(v^0_n) from v^0_{N_tau} = 0) into Gk (and Gk_th), each solve
//    from its input; k_cm_guess then prolongs it into the fine guesses.
// After a correction launch, k_cm_correct forms the corrected fine states
// F_n + P(Gn[n] - Gk[n]) and k_cm_sens the coarse-correction sensitivities.
//
// Every solve is Jacobi PCG in the single-reduction form of Chronopoulos and
// Gear, one group barrier per iteration, on the assembled 9-point rows of
// C_c/dtau + K_c. The group's workgroups own contiguous coarse-node tiles; each
// round stages the z window of its tile (one coarse row plus one node of halo
// each side) in LDS, forming the halo z pointwise from the neighbours' r, w, s
// of the previous round. The vectors live in the group's pool slots and move
// between workgroups with device-coherent loads and stores. CG stops on the
// recursive residual; the true residual b - A x then decides (at most three
// restarts from it), as in the engine's fine solves. Reductions are in a
// fixed order.

// Coarse node I's fine node.
__device__ __forceinline__ int cml_fine(const Consts &C, const CoarseMesh &M, int I) {
    const int J = I / M.Wc, i = I - J * M.Wc;
    return 2 * J * C.W + 2 * i;
}

// Row of S holding the fine state T_j (store-all, or the checkpointed slice
// ends T_{Mn} and slice starts T_{Mn+1}: the only states these lanes read).
__device__ __forceinline__ const double *cml_srow(const Consts &C, const Bufs &B, int j) {
    if (!C.ckpt) return B.S + (size_t)(j - 1) * C.Nn;
    if (j % C.M == 0) return B.S + (size_t)(j / C.M - 1) * C.Nn;
    return B.S + (size_t)(C.Ntau + (j - 1) / C.M) * C.Nn;
}

// 9-point row I (entry k = (dj+1)*3 + (di+1)) applied to a window holding
// coarse node I at index li. Entries towards missing neighbours (mesh edges,
// Dirichlet columns) are zero, so the wrapped window values there do not count.
__device__ __forceinline__ double cml_row(const double *S9, int Nc, int I, const double *Wn, int li,
                                          int Wc) {
    const double *r = S9 + I;
    const size_t s = (size_t)Nc;
    return r[0] * Wn[li - Wc - 1] + r[s] * Wn[li - Wc] + r[2 * s] * Wn[li - Wc + 1] +
           r[3 * s] * Wn[li - 1] + r[4 * s] * Wn[li] + r[5 * s] * Wn[li + 1] +
           r[6 * s] * Wn[li + Wc - 1] + r[7 * s] * Wn[li + Wc] + r[8 * s] * Wn[li + Wc + 1];
}

// (P x)_id at fine node id, x a coarse vector written in this launch.
__device__ __forceinline__ double cml_prolong(const Consts &C, const CoarseMesh &M,
                                              const unsigned char *mask, const double *x, int id) {
    if (mask[id]) return 0.0;
    const int j = id / C.W, i = id - j * C.W;
    const double *r0 = x + (size_t)(j >> 1) * M.Wc + (i >> 1);
    if (!(i & 1) && !(j & 1)) return ldc(r0);
    if (!(j & 1)) return 0.5 * ldc(r0) + 0.5 * ldc(r0 + 1);
    if (!(i & 1)) return 0.5 * ldc(r0) + 0.5 * ldc(r0 + M.Wc);
    return 0.25 * ldc(r0) + 0.25 * ldc(r0 + 1) + 0.25 * ldc(r0 + M.Wc) +
           0.25 * ldc(r0 + M.Wc + 1);
}

// (P^T s)_I for the fine adjoint source s = scale T^{o(p-1)} (Eq. 4.6), with
// the bilinear weights 1, 1/2, 1/4 of the fine nodes around coarse node I.
__device__ __forceinline__ double cml_source(const Consts &C, const CoarseMesh &M,
                                             const unsigned char *mask, const double *Tm,
                                             double scale, int I) {
    const int J = I / M.Wc, i = I - J * M.Wc;
    double s = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int fj = 2 * J + dj;
        if (fj < 0 || fj > C.ny) continue;
        for (int di = -1; di <= 1; ++di) {
            const int fi = 2 * i + di;
            if (fi < 0 || fi > C.nx) continue;
            const int id = fj * C.W + fi;
            if (mask[id]) continue;
            const double w = (di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5);
            s += w * (scale * ipow(Tm[id], C.p - 1));
        }
    }
    return s;
}

// Group reduction of Q partial sums: this workgroup's block sum goes to its
// partial slot (by barrier parity), the group barrier, then every workgroup
// sums the slots in the same order.
template <int Q>
__device__ __forceinline__ bool cml_reduce(double (&v)[Q], double *red, double *part, int rank,
                                           int g, unsigned *bar, unsigned &nbar, Control *ctl,
                                           long long tmo, bool release) {
    block_sum<Q>(v, red);
    const int par = nbar & 1;
    if (threadIdx.x == 0)
        for (int q = 0; q < Q; ++q) stc(part + ((size_t)par * kMaxGroup + rank) * 4 + q, v[q]);
    ++nbar;
    if (!group_barrier<false>(bar, (unsigned)g, nbar * (unsigned)g, ctl, tmo, release))
        return false;
    group_sum<Q>(part + (size_t)par * kMaxGroup * 4, g, v, red);
    return true;
}

// Runs one coarse-mesh lane (kind CM_*, slice `slice`) of the design whose
// descriptor is Ed on this workgroup's group: `rank` of `g` workgroups, group
// barrier counter `bar` after `nbar` barriers, partial-sum slots `part`, group
// vector set `vec`. Returns the group's barrier count after the lane, or -1
// when a wait timed out or another workgroup aborted (every workgroup of the
// group returns alike). `trec`: the lane's trace record, `trace_steps` the
// step timestamps it holds. Dynamic LDS: 2 (ceil(Nc/g) + 2 (Wc + 1)) doubles.
__device__ __forceinline__ long long cm_lane(const EngineDesc *__restrict__ Ed, int kind, int slice,
                                          int rank, int g, int vec, unsigned *bar, double *part,
                                          unsigned nbar, unsigned long long *trec,
                                          int trace_steps) {
    extern __shared__ double cml_lds[];
    __shared__ double red[kWaves * 4];
    const Consts &C = Ed->C;
    const Bufs &B = Ed->B;
    const CoarseMesh &M = Ed->cm;
    const LaunchInfo &I = Ed->I;
    Control *ctl = B.ctl;
    const long long tmo = C.timeout_ticks;
    const bool adj = kind == CM_GK_ADJ || kind == CM_SWEEP_ADJ;
    const bool sweep = kind == CM_SWEEP_PRI || kind == CM_SWEEP_ADJ;
    const bool cold = sweep && I.cold;  // the cold coarse sweep
    const int Nc = M.Nc, Wc = M.Wc, Hc = Wc + 1;
    const int ts = (Nc + g - 1) / g;
    const int a = min(rank * ts, Nc), b = min(a + ts, Nc);
    const int lo = a - Hc, len = (b - a) + 2 * Hc;
    double *W0 = cml_lds;                // staged window: u, or z of a round
    double *W1 = cml_lds + ts + 2 * Hc;  // second window: x0 / x, or r of a round
    double *U = group_vec(B, vec, V_TP);   // the step's coarse input u
    double *Bv = group_vec(B, vec, V_TQ);  // right-hand side b
    double *P = group_vec(B, vec, V_P);
    double *Rv[2] = {group_vec(B, vec, V_R0), group_vec(B, vec, V_R1)};
    double *Wv[2] = {group_vec(B, vec, V_W0), group_vec(B, vec, V_W1)};
    double *Sv[2] = {group_vec(B, vec, V_S0), group_vec(B, vec, V_S1)};
    const bool leader = rank == 0 && threadIdx.x == 0;
    const unsigned nbar0 = nbar;
    unsigned long long iters_all = 0;
    const int Nt = C.Ntau;
    // a batched lane is one step of slice `slice`; the primal correction sweep
    // runs n = 1 .. N_tau-1, the adjoint one n = N_tau-1 .. 1; the cold sweeps
    // n = 0 .. N_tau-1 and n = N_tau .. 1
    const int nsteps = cold ? Nt : sweep ? Nt - 1 : 1;
    if (leader) {
        trec[TR_KIND] = kind;
        trec[TR_SLICE] = slice;
        trec[TR_NWG] = g;
        trec[TR_TILE] = ts;
        trec[TR_START] = (unsigned long long)now_ticks();
    }
    auto barrier = [&](bool rel) {
        ++nbar;
        return group_barrier<false>(bar, (unsigned)g, nbar * (unsigned)g, ctl, tmo, rel);
    };
    auto waitf = [&](int fk, int n) {
        return wait_flag(B.flags, flag_index(fk, n), I.epoch, ctl, tmo);
    };
    // the adjoint source factor Theta^{1-p}/N_e (Eq. 4.6)
    const double scale = adj ? pow_call(*B.Theta, 1.0 - C.p) / (double)C.Ne : 0.0;

    // the correction sweep's first input R F_0 (primal) or R F_{N_tau}
    // (adjoint); the cold sweep's is 0
    double theta = 0.0;
    if (cold) {
        for (int q = a + threadIdx.x; q < b; q += kThreads) stc(U + q, 0.0);
        if (!barrier(false)) return -1;
    } else if (sweep) {
        if (!waitf(FL_F, adj ? Nt : 0)) return -1;
        const double *F0 = adj ? B.FL + (size_t)Nt * C.Nn : cml_srow(C, B, C.M);
        for (int q = a + threadIdx.x; q < b; q += kThreads)
            stc(U + q, M.dinv[q] == 0.0 ? 0.0 : ldc(F0 + cml_fine(C, M, q)));
        if (!adj) {
            theta = B.F_th[0];
            if (leader) B.out_th[1] = theta;
        }
        if (!barrier(false)) return -1;
    }
    for (int step = 0; step < nsteps; ++step) {
        const int n = cold ? (adj ? Nt - step : step)
                           : sweep ? (adj ? Nt - 1 - step : step + 1) : slice;
        const double *Tm = adj ? cml_srow(C, B, C.M * (n - 1) + 1) : nullptr;
        const double qn = adj ? 0.0 : B.qt[C.M * (n + 1)];
        double *X = (sweep && !cold ? M.Gn : M.Gk) + (size_t)n * Nc;  // the step's output
        const double *gk = M.Gk + (size_t)n * Nc;
        // u^k_n (no guess in the cold sweep)
        const double *fin = cold ? nullptr : (adj ? B.in_L : B.in_T) + (size_t)n * C.Nn;
        if (sweep && !cold && I.gk_lanes && !waitf(FL_GK, n)) return -1;
        double bnorm = 0.0, rn = 0.0, alpha = 0.0, beta = 0.0, gamma = 0.0;
        int iter = 0, restarts = 0;
        bool verify = false;
        for (;;) {
            // INIT: b = C_c/dtau u + load and x0 (a sweep step starts from
            // G(R u^k_n) + (u - R u^k_n)); verification passes keep b and x.
            // Then r0 = b - A x0, with ||b|| and ||r0||.
            lds_sync();
            for (int q = threadIdx.x; q < len; q += kThreads) {
                const int id = lo + q;
                double u = 0.0, x0 = 0.0;
                if (id >= 0 && id < Nc && M.dinv[id] != 0.0) {
                    if (verify) {
                        x0 = ldc(X + id);
                    } else if (cold) {
                        u = ldc(U + id);
                        x0 = u;
                    } else {
                        const double rk = fin[cml_fine(C, M, id)];
                        u = sweep ? ldc(U + id) : rk;
                        x0 = sweep ? ldc(gk + id) + (u - rk) : u;
                    }
                }
                W0[q] = u;
                W1[q] = x0;
            }
            lds_sync();
            double l2[2] = {0.0, 0.0};
            for (int id = a + threadIdx.x; id < b; id += kThreads) {
                const int li = id - lo;
                double bb = 0.0, r0 = 0.0;
                if (M.dinv[id] != 0.0) {
                    if (verify) {
                        bb = ldc(Bv + id);
                    } else {
                        const double load = adj ? cml_source(C, M, B.mask, Tm, scale, id)
                                                : qn * M.fc[id];
                        bb = cml_row(M.C9, Nc, id, W0, li, Wc) + load;
                    }
                    r0 = bb - cml_row(M.A9, Nc, id, W1, li, Wc);
                }
                if (!verify) {
                    stc(Bv + id, bb);
                    stc(X + id, W1[li]);
                }
                stc(Rv[0] + id, r0);
                l2[0] += bb * bb;
                l2[1] += r0 * r0;
            }
            if (!cml_reduce<2>(l2, red, part, rank, g, bar, nbar, ctl, tmo, false)) return -1;
            if (!verify) bnorm = sqrt(l2[0]);
            rn = sqrt(l2[1]);
            if (bnorm == 0.0) {
                // b = 0: x = 0
                for (int id = a + threadIdx.x; id < b; id += kThreads) stc(X + id, 0.0);
                rn = 0.0;
                if (!barrier(false)) return -1;
                break;
            }
            if (rn <= C.rtol * bnorm) break;
            if (verify && (restarts >= 3 || iter >= C.max_iter)) break;
            if (verify) ++restarts;
            // FIRST: z0 = D^{-1} r0, w0 = A z0; gamma = (r0, z0), delta = (z0, w0)
            lds_sync();
            for (int q = threadIdx.x; q < len; q += kThreads) {
                const int id = lo + q;
                double r = 0.0, z = 0.0;
                if (id >= 0 && id < Nc) {
                    r = ldc(Rv[0] + id);
                    z = M.dinv[id] * r;
                }
                W0[q] = z;
                W1[q] = r;
            }
            lds_sync();
            double f2[2] = {0.0, 0.0};
            for (int id = a + threadIdx.x; id < b; id += kThreads) {
                const int li = id - lo;
                const double z = W0[li];
                const double w = M.dinv[id] == 0.0 ? 0.0 : cml_row(M.A9, Nc, id, W0, li, Wc);
                stc(Wv[0] + id, w);
                f2[0] += W1[li] * z;
                f2[1] += z * w;
            }
            if (!cml_reduce<2>(f2, red, part, rank, g, bar, nbar, ctl, tmo, false)) return -1;
            gamma = f2[0];
            alpha = f2[0] / f2[1];
            beta = 0.0;
            // ITER (one reduction per round): s = w + beta s, r' = r - alpha s,
            // p = z + beta p, x += alpha p, z' = D^{-1} r', w' = A z'
            for (int il = 0;; ++il) {
                const int cur = il & 1, nxt = cur ^ 1;
                const bool first = il == 0;
                lds_sync();
                for (int q = threadIdx.x; q < len; q += kThreads) {
                    const int id = lo + q;
                    double z = 0.0, rnew = 0.0;
                    if (id >= 0 && id < Nc) {
                        const double d = M.dinv[id];
                        const double r = ldc(Rv[cur] + id), w = ldc(Wv[cur] + id);
                        const double sn = first ? w : w + beta * ldc(Sv[cur] + id);
                        rnew = r - alpha * sn;
                        z = d * rnew;
                        if (id >= a && id < b) {
                            const double pn = first ? d * r : d * r + beta * ldc(P + id);
                            stc(P + id, pn);
                            stc(X + id, ldc(X + id) + alpha * pn);
                            stc(Sv[nxt] + id, sn);
                            stc(Rv[nxt] + id, rnew);
                        }
                    }
                    W0[q] = z;
                    W1[q] = rnew;
                }
                lds_sync();
                double l3[3] = {0.0, 0.0, 0.0};
                for (int id = a + threadIdx.x; id < b; id += kThreads) {
                    const int li = id - lo;
                    const double z = W0[li], r = W1[li];
                    const double w = M.dinv[id] == 0.0 ? 0.0 : cml_row(M.A9, Nc, id, W0, li, Wc);
                    stc(Wv[nxt] + id, w);
                    l3[0] += r * z;
                    l3[1] += z * w;
                    l3[2] += r * r;
                }
                if (!cml_reduce<3>(l3, red, part, rank, g, bar, nbar, ctl, tmo, false)) return -1;
                ++iter;
                rn = sqrt(l3[2]);
                if (rn <= C.rtol * bnorm || iter >= C.max_iter) break;
                const double bnew = l3[0] / gamma;
                alpha = l3[0] / (l3[1] - bnew * l3[0] / alpha);
                beta = bnew;
                gamma = l3[0];
            }
            verify = true;  // the true residual of x decides
        }
        iters_all += iter;
        // POST: the next input of a sweep, u = x + R F_n - G(R u^k_n), or x
        // in the cold sweep
        if (cold) {
            for (int id = a + threadIdx.x; id < b; id += kThreads) stc(U + id, ldc(X + id));
        } else if (sweep) {
            if (!waitf(FL_F, n)) return -1;
            const double *Fn = adj ? B.FL + (size_t)n * C.Nn : cml_srow(C, B, C.M * (n + 1));
            for (int id = a + threadIdx.x; id < b; id += kThreads)
                stc(U + id, M.dinv[id] == 0.0
                                ? 0.0
                                : ldc(X + id) + ldc(Fn + cml_fine(C, M, id)) - ldc(gk + id));
        }
        // primal theta (Alg. 1 with dtau, N_tau) from ||P x||_p^p over the fine nodes
        double th[1] = {0.0};
        if (!adj) {
            const int fts = (C.Nn + g - 1) / g;
            const int fa = min(rank * fts, C.Nn), fb = min(fa + fts, C.Nn);
            for (int id = fa + threadIdx.x; id < fb; id += kThreads)
                th[0] += ipow(cml_prolong(C, M, B.mask, X, id), C.p);
            // release: the outputs become visible to the lanes that wait on this one
            if (!cml_reduce<1>(th, red, part, rank, g, bar, nbar, ctl, tmo, true)) return -1;
        } else if (!barrier(true)) {
            return -1;
        }
        if (!adj) {
            const double base = sweep ? theta : B.in_th[n];
            const double thG = pow_call(ipow(base, C.p) + th[0] * C.inv_NtauNe, C.inv_p);
            if (cold) {
                theta = thG;
                if (leader) B.Gk_th[n] = thG;
            } else if (sweep) {
                theta = thG + B.F_th[n] - B.Gk_th[n];
                if (leader) {
                    B.Gn_th[n] = thG;
                    B.out_th[n + 1] = theta;
                }
            } else if (leader) {
                B.Gk_th[n] = thG;
            }
        }
        if (leader) {
            const double rr = bnorm > 0.0 ? rn / bnorm : 0.0;
            atomicAdd(&ctl->iters_coarse, (unsigned long long)iter);
            atomicAdd(&ctl->solves_coarse, 1ull);
            atomicMax(&ctl->max_iters, iter);
            atomicMax(&ctl->max_relres_bits, (unsigned long long)__double_as_longlong(rr));
            if (!isfinite(rr)) set_status(ctl, -5);
            else if (bnorm > 0.0 && !(rn <= C.rtol * bnorm)) set_status(ctl, -4);
            if (!sweep) set_flag(B.flags, flag_index(FL_GK, n), I.epoch);
            if (step < trace_steps) trec[TR_HDR + step] = (unsigned long long)now_ticks();
        }
    }
    if (leader) {
        trec[TR_ROUNDS] = nbar - nbar0;
        trec[TR_ITERS] = iters_all;
    }
    return (long long)nbar;
}
