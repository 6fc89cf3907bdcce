// Coupling geometry of the operator, built once per problem (independent of
// the energy and of the right-hand sides).
//
// The coupling term of component alpha at a collocation point needs both
// partners' expansions at the point's image in the partner's Jacobi
// coordinates (the rotation of Sec. 2 between Jacobi sets, with the cosine of
// the angle from the relation between the two triangles).  For every point
// with a nonzero short-range potential and every partner beta whose box holds
// the image, this records the spline cell of beta that contains the image, the
// image's position inside that cell (0..1 per dimension), and the n_M x n_M
// factor that multiplies beta's values there: V_alpha^(s) x y / (x_beta y_beta)
// times, for L > 0, the Wigner-function weights between the M' blocks
// (eq. (FM-pre)).  The pairs are grouped by (beta, cell) and the groups are cut
// into tasks of at most 64 pairs: a wave evaluates one task from one cell's
// coefficients.
#include <algorithm>
#include <cmath>
#include <thread>

#include "fm_problem.h"

namespace fm {

namespace {

bool cyclic(int b, int a) { return (b == 0 && a == 1) || (b == 1 && a == 2) || (b == 2 && a == 0); }

struct Rec {
    int key;
    int out;
    double s[3];
};

}  // namespace

std::string build_coupling(const fm_problem *p, const HostFactors &hf, CouplingHost &ch) {
    const int nM = p->nM, J = p->desc.J, M0 = p->M0;
    const int nf = nM * nM;
    const ProblemDev &pd = p->pd;
    int keyoff[4] = {0, 0, 0, 0};
    for (int b = 0; b < 3; ++b) keyoff[b + 1] = keyoff[b] + p->bz[b].K * p->bx[b].K * p->by[b].K;

    // one work item per (alpha, z point); each thread keeps its own records
    struct Item { int a, iz; };
    std::vector<Item> items;
    for (int a = 0; a < 3; ++a)
        if (!p->absent(a))
            for (int iz = 0; iz < p->bz[a].n; ++iz) items.push_back({a, iz});
    const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::vector<Rec>> recs(nth);
    std::vector<std::vector<double>> facs(nth);
    auto work = [&](int t) {
        for (size_t it = t; it < items.size(); it += nth) {
            const int a = items[it].a, iz = items[it].iz;
            const Basis1D &ax = p->bx[a], &ay = p->by[a], &az = p->bz[a];
            const int nx = ax.n, ny = ay.n;
            const double zc = az.points[iz], omz = 1.0 - zc * zc;
            const std::vector<double> &Vs = hf.comp[a].Vs;
            for (int ix = 0; ix < nx; ++ix)
                for (int iy = 0; iy < ny; ++iy) {
                    const double vs = Vs[size_t(ix) * ny + iy];
                    if (vs == 0.0) continue;
                    const double xc = ax.points[ix], yc = ay.points[iy];
                    for (int bb = 0; bb < 2; ++bb) {
                        const int b = (a + 1 + bb) % 3;
                        // exchange-reduced problems: partner 2 is p (-1)^{M''} times partner 1
                        // at -z (eq. (2-sym-part)); with three identical particles both partners
                        // are component 1 itself in their own coordinates (eq. (3-sym-part)).
                        // The cell is looked up in component 1
                        const bool implied = p->absent(b);
                        const bool mirror = implied && p->exchange != 3;
                        const int bc = implied ? 0 : b;
                        const Basis1D &bx = p->bx[bc], &by = p->by[bc], &bz = p->bz[bc];
                        const double c = p->crot[b][a], s = p->srot[b][a];
                        const double xb =
                            std::sqrt(std::fmax(c * c * xc * xc + 2.0 * s * c * xc * yc * zc + s * s * yc * yc, 0.0));
                        const double yb =
                            std::sqrt(std::fmax(s * s * xc * xc - 2.0 * s * c * xc * yc * zc + c * c * yc * yc, 0.0));
                        if (!(xb <= bx.nodes.back() && yb <= by.nodes.back())) continue;
                        const double den = xb * yb;
                        double zb = den > 0.0 ? (s * c * (yc * yc - xc * xc) + (c * c - s * s) * xc * yc * zc) / den
                                              : 0.0;
                        zb = std::fmin(1.0, std::fmax(-1.0, zb));
                        double zl = mirror ? -zb : zb;                // where the stored component is read
                        // component 3 stored on z in [0, 1] (zhalf): read at |z| times its parity
                        double fold = 1.0;
                        if (p->zhalf && bc == 2 && zl < 0.0) {
                            zl = -zl;
                            fold = p->zsigma;
                        }
                        const int mz = bz.interval(zl), mx = bx.interval(xb), my = by.interval(yb);
                        Rec r;
                        r.key = keyoff[bc] + (mz * bx.K + mx) * by.K + my;
                        r.out = int((p->off[a] + (long long)(iz * nx + ix) * ny + iy) * 2 + bb);
                        r.s[0] = (zl - bz.nodes[mz]) / (bz.nodes[mz + 1] - bz.nodes[mz]);
                        r.s[1] = (xb - bx.nodes[mx]) / (bx.nodes[mx + 1] - bx.nodes[mx]);
                        r.s[2] = (yb - by.nodes[my]) / (by.nodes[my + 1] - by.nodes[my]);
                        recs[t].push_back(r);
                        const double base = vs * xc * yc / den;
                        if (J == 0) {
                            facs[t].push_back((mirror ? p->exchange * base : base) * fold);
                            continue;
                        }
                        double arg = (-s * xc * zc + c * yc) / yb;
                        arg = std::fmin(1.0, std::fmax(-1.0, arg));
                        double cw = std::sqrt(0.5 * (1.0 + arg)), sw = std::sqrt(0.5 * (1.0 - arg));
                        if (!cyclic(b, a)) cw = -cw;
                        const double sa = std::sqrt(std::fmax(omz, 0.0)), sb = std::sqrt(std::fmax(1.0 - zb * zb, 0.0));
                        double sbp[MAXM], sap[MAXM];
                        sbp[0] = M0 ? sb : 1.0;
                        sap[0] = M0 ? sa : 1.0;
                        for (int k = 1; k < nM; ++k) {
                            sbp[k] = sbp[k - 1] * sb;
                            sap[k] = sap[k - 1] * sa;
                        }
                        for (int iM = 0; iM < nM; ++iM)
                            for (int jM = 0; jM < nM; ++jM) {
                                const double *G = pd.dcoef + (iM * nM + jM) * pd.dlen;
                                // sum_k G[k] cw^k sw^(2J-k) by Horner in cw
                                double f = G[2 * J], sp = 1.0;
                                for (int k = 2 * J - 1; k >= 0; --k) {
                                    sp *= sw;
                                    f = f * cw + G[k] * sp;
                                }
                                double w = base * f * sbp[jM] / sap[iM];
                                if (mirror) w *= p->exchange * (((M0 + jM) & 1) ? -1.0 : 1.0);
                                facs[t].push_back(w * fold);
                            }
                    }
                }
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(work, t);
    for (auto &x : th) x.join();

    // counting sort by cell (stable within a cell: alpha order)
    long long np = 0;
    for (auto &v : recs) np += (long long)v.size();
    if (np >= (1LL << 31)) return "too many coupling pairs";
    std::vector<long long> start(keyoff[3] + 1, 0);
    for (auto &v : recs)
        for (const Rec &r : v) start[r.key + 1]++;
    for (int k = 0; k < keyoff[3]; ++k) start[k + 1] += start[k];
    std::vector<long long> pos(start.begin(), start.end() - 1);
    ch.npairs = np;
    ch.out.assign(np, 0);
    ch.s.assign(3 * np, 0.0);
    ch.F.assign(size_t(nf) * np, 0.0);
    // each thread holds its items' records in item order; walking the items in
    // order and taking each one's records from its thread keeps alpha order
    {
        std::vector<size_t> ri(nth, 0);
        for (size_t it = 0; it < items.size(); ++it) {
            const int t = int(it % nth);
            const int a = items[it].a, iz = items[it].iz;
            const long long lo = p->off[a] + (long long)iz * p->bx[a].n * p->by[a].n;
            const long long hi = lo + (long long)p->bx[a].n * p->by[a].n;
            while (ri[t] < recs[t].size()) {
                const Rec &r = recs[t][ri[t]];
                const long long o = r.out >> 1;
                if (o < lo || o >= hi) break;
                const long long d = pos[r.key]++;
                ch.out[d] = r.out;
                for (int k = 0; k < 3; ++k) ch.s[size_t(k) * np + d] = r.s[k];
                for (int f = 0; f < nf; ++f) ch.F[size_t(f) * np + d] = facs[t][ri[t] * nf + f];
                ++ri[t];
            }
        }
        for (int t = 0; t < nth; ++t)
            if (ri[t] != recs[t].size()) return "coupling pair merge failed";
    }
    // tasks: (beta, cell) groups cut into chunks of at most 64 pairs, each with
    // the cell's function indices and beta's sizes
    ch.task.clear();
    ch.r.clear();
    for (int b = 0; b < 3; ++b) {
        const Basis1D &bz = p->bz[b], &bx = p->bx[b], &by = p->by[b];
        const int Kz = bz.K, Kx = bx.K, Ky = by.K;
        for (int mz = 0; mz < Kz; ++mz)
            for (int mx = 0; mx < Kx; ++mx)
                for (int my = 0; my < Ky; ++my) {
                    const int key = keyoff[b] + (mz * Kx + mx) * Ky + my;
                    for (long long q = start[key]; q < start[key + 1]; q += 64) {
                        int rec[CPL_TASK] = {};
                        rec[CT_BETA] = b;
                        rec[CT_MZ] = mz;
                        rec[CT_MX] = mx;
                        rec[CT_MY] = my;
                        rec[CT_FIRST] = int(q);
                        rec[CT_COUNT] = int(std::min<long long>(64, start[key + 1] - q));
                        rec[CT_NX] = bx.n;
                        rec[CT_NY] = by.n;
                        rec[CT_NPTS] = int(p->npts[b]);
                        const unsigned long long off = (unsigned long long)p->off[b];
                        rec[CT_OFF_LO] = int(off & 0xffffffffull);
                        rec[CT_OFF_HI] = int(off >> 32);
                        rec[CT_TASK] = int(ch.task.size() / CPL_TASK);
                        int *f = rec + CT_FIDX;
                        for (int k = 0; k < 2 * bz.q; ++k) *f++ = bz.global_index(mz + k / bz.q, k % bz.q);
                        for (int k = 0; k < 2 * bx.q; ++k) *f++ = bx.global_index(mx + k / bx.q, k % bx.q);
                        for (int k = 0; k < 2 * by.q; ++k) *f++ = by.global_index(my + k / by.q, k % by.q);
                        ch.task.insert(ch.task.end(), rec, rec + CPL_TASK);
                        ch.r.push_back((bz.nodes[mz + 1] - bz.nodes[mz]) / bz.hbar);
                        ch.r.push_back((bx.nodes[mx + 1] - bx.nodes[mx]) / bx.hbar);
                        ch.r.push_back((by.nodes[my + 1] - by.nodes[my]) / by.hbar);
                    }
                }
    }
    ch.ntasks = int(ch.task.size() / CPL_TASK);
    // wave jobs.  With one M'' block, two consecutive tasks (neighbouring cells)
    // share a wave, one per half: when the tasks average more than 40 pairs,
    // every two, with up to two pairs per lane (each staged coefficient then
    // feeds two products); otherwise two of at most 32 pairs, one pair per lane
    // (fewer registers; cells with few pairs still fill a wave).  With more M''
    // blocks, one task per wave.
    ch.job.clear();
    ch.pairs_per_lane = (nM == 1 && ch.ntasks > 0 && np > 40LL * ch.ntasks) ? 2 : 1;
    auto cnt = [&](int t) { return ch.task[size_t(t) * CPL_TASK + CT_COUNT]; };
    for (int t = 0; t < ch.ntasks; ++t) {
        ch.job.push_back(t);
        const bool pair = nM == 1 && t + 1 < ch.ntasks &&
                          (ch.pairs_per_lane == 2 || (cnt(t) <= 32 && cnt(t + 1) <= 32));
        if (pair) {
            ch.job.push_back(t + 1);
            ++t;
        } else {
            ch.job.push_back(-1);
        }
    }
    ch.njobs = int(ch.job.size() / 2);
    // job-ordered records (one M'' block): each half's own task record; a job
    // of one task repeats it in the second half (unsplit) or, when every job is
    // split, leaves that half empty.  More M'' blocks: job j must be task j.
    ch.jrec.clear();
    if (nM == 1) {
        ch.jrec.assign(size_t(ch.njobs) * 2 * CPL_TASK, 0);
        for (int j = 0; j < ch.njobs; ++j) {
            const int t0 = ch.job[2 * j], t1 = ch.job[2 * j + 1];
            const bool split = t1 >= 0;
            int *r0 = &ch.jrec[size_t(2 * j) * CPL_TASK], *r1 = r0 + CPL_TASK;
            std::copy_n(&ch.task[size_t(t0) * CPL_TASK], CPL_TASK, r0);
            if (split) {
                std::copy_n(&ch.task[size_t(t1) * CPL_TASK], CPL_TASK, r1);
            } else if (ch.pairs_per_lane == 1) {
                std::copy_n(r0, CPL_TASK, r1);
            } else {
                r1[CT_TASK] = -1;               // count 0: no pairs
                r1[CT_SPLIT] = 1;
            }
            r0[CT_SPLIT] = split ? 1 : 0;
            if (split || ch.pairs_per_lane == 1) r1[CT_SPLIT] = r0[CT_SPLIT];
        }
    } else {
        for (int j = 0; j < ch.njobs; ++j)
            if (ch.job[2 * j] != j || ch.job[2 * j + 1] != -1) return "coupling jobs out of task order";
        if (ch.njobs != ch.ntasks) return "coupling jobs out of task order";
    }
    return "";
}

}  // namespace fm
